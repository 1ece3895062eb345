// 12-6 Lennard-Jones forces, energy and virial over a Verlet list.
//
// Sec. 4, Eq. (1): E = sum over pairs with r < r_c of 4 eps [(s/r)^12 - (s/r)^6]
// (truncated, not shifted); the force on i is the pairwise sum of -dU/dr
// along d = x_i - x_j.  With r2i = 1/r^2 and r6i = r2i^3:
//   fpair = r6i (lj1 r6i - lj2) r2i,  lj1 = 48 eps s^12, lj2 = 24 eps s^6
//   U     = r6i (lj3 r6i - lj4),      lj3 =  4 eps s^12, lj4 =  4 eps s^6
// Sec. 4.1 gives the two schemes:
//   - full list, "gather": one atom per lane, every pair computed twice, no
//     atomics; E and W take half of each entry;
//   - half list, "scatter": each pair once, the partner's force added with
//     FP64 atomics.
// The mixed-precision variant keeps positions, displacement, r^2 and the
// cutoff test in FP64 and evaluates the pair terms (r2i, r6i, fpair, U) in
// FP32; forces, energy and virial accumulate in FP64.
#include "tile.hpp"

#include <algorithm>

namespace ljmd {

namespace {

constexpr int kThreads = 256;

struct ForceArgs {
    const double *x;
    const int32_t *type;
    int64_t n;
    Box box;
    const int32_t *numneigh;
    const uint32_t *neigh;
    int cap;
    double *f;
    double *partials;  // [blocks][kPartVals] when energy/virial requested
};

// Displacement x_i - x_j with the image stored in the list entry.
__device__ __forceinline__ void apply_image(uint32_t code, const Box &box, double &dx,
                                            double &dy, double &dz) {
    if (code & 1u) dx -= box.L[0];
    else if (code & 2u) dx += box.L[0];
    if (code & 4u) dy -= box.L[1];
    else if (code & 8u) dy += box.L[1];
    if (code & 16u) dz -= box.L[2];
    else if (code & 32u) dz += box.L[2];
}

// FP64 reciprocal: the hardware estimate (relative error below 5e-8 on
// gfx950) refined by one Newton step (e = 1 - a y, y += y e), which squares
// the error to a few 1e-15, a few ulp; the forces stay far inside the 1e-12
// parity bound.
__device__ __forceinline__ double recip(double a) {
    const double y = __builtin_amdgcn_rcp(a);
    return fma(y, fma(-a, y, 1.0), y);
}

struct Coef {
    double rc2, lj1, lj2, lj3, lj4;
    float lj1f, lj2f, lj3f, lj4f;
};

// Per-type-pair lookup: T == 1 reads the uniform kernel arguments, T > 1 the
// copy staged in LDS.
struct CoefLds {
    double rc2[kTab], lj1[kTab], lj2[kTab], lj3[kTab], lj4[kTab];
    float lj1f[kTab], lj2f[kTab], lj3f[kTab], lj4f[kTab];
};

__device__ __forceinline__ void stage_coef(CoefLds &c, const PairTab &t) {
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kTab; ++k) {
            c.rc2[k] = t.rc2[k];
            c.lj1[k] = t.lj1[k];
            c.lj2[k] = t.lj2[k];
            c.lj3[k] = t.lj3[k];
            c.lj4[k] = t.lj4[k];
            c.lj1f[k] = t.lj1f[k];
            c.lj2f[k] = t.lj2f[k];
            c.lj3f[k] = t.lj3f[k];
            c.lj4f[k] = t.lj4f[k];
        }
    }
    __syncthreads();
}

template <int T>
__device__ __forceinline__ Coef get_coef(const CoefLds &c, const PairTab &t, int k) {
    Coef r;
    if (T == 1) {
        r.rc2 = t.rc2[0];
        r.lj1 = t.lj1[0];
        r.lj2 = t.lj2[0];
        r.lj3 = t.lj3[0];
        r.lj4 = t.lj4[0];
        r.lj1f = t.lj1f[0];
        r.lj2f = t.lj2f[0];
        r.lj3f = t.lj3f[0];
        r.lj4f = t.lj4f[0];
    } else {
        r.rc2 = c.rc2[k];
        r.lj1 = c.lj1[k];
        r.lj2 = c.lj2[k];
        r.lj3 = c.lj3[k];
        r.lj4 = c.lj4[k];
        r.lj1f = c.lj1f[k];
        r.lj2f = c.lj2f[k];
        r.lj3f = c.lj3f[k];
        r.lj4f = c.lj4f[k];
    }
    return r;
}

// Pair force magnitude over r (fpair) and, if wanted, the pair energy.
template <bool MIXED, bool EV>
__device__ __forceinline__ void pair_terms(double rsq, const Coef &c, double &fpair,
                                           double &u) {
    if (MIXED) {
        const float r2i = __builtin_amdgcn_rcpf((float)rsq);
        const float r6i = r2i * r2i * r2i;
        fpair = (double)(r6i * (c.lj1f * r6i - c.lj2f) * r2i);
        if (EV) u = (double)(r6i * (c.lj3f * r6i - c.lj4f));
    } else {
        const double r2i = recip(rsq);
        const double r6i = r2i * r2i * r2i;
        fpair = r6i * fma(c.lj1, r6i, -c.lj2) * r2i;
        if (EV) u = r6i * fma(c.lj3, r6i, -c.lj4);
    }
}

// Sum per-lane values over the block in a fixed order and store one row of
// partials for this block.
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double *out) {
    __shared__ double s[kThreads / kWave][NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) s[threadIdx.x >> 6][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
        for (int w = 0; w < kThreads / kWave; ++w) t += s[w][threadIdx.x];
        out[threadIdx.x] = t;
    }
}

template <int T, bool EV, bool MIXED>
__global__ __launch_bounds__(kThreads) void k_force_gather(ForceArgs a, PairTab tab) {
    __shared__ CoefLds cl;
    if (T > 1) stage_coef(cl, tab);
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t i = blk * kThreads + threadIdx.x;
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    if (i < a.n) {
        const double xi = a.x[3 * i], yi = a.x[3 * i + 1], zi = a.x[3 * i + 2];
        const int ti = T > 1 ? a.type[i] : 0;
        const int nn = a.numneigh[i];
        const uint32_t *row = a.neigh + ((i >> 6) * (int64_t)a.cap) * kWave + (i & 63);
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int k = 0; k < nn; ++k) {
            const uint32_t raw = row[(int64_t)k * kWave];
            const int64_t j = raw & kIndexMask;
            double dx = xi - a.x[3 * j];
            double dy = yi - a.x[3 * j + 1];
            double dz = zi - a.x[3 * j + 2];
            const uint32_t code = raw >> kCodeShift;
            if (code) apply_image(code, a.box, dx, dy, dz);
            const double rsq = fma(dz, dz, fma(dy, dy, dx * dx));
            const int tj = T > 1 ? a.type[j] : 0;
            const Coef c = get_coef<T>(cl, tab, ti * T + tj);
            if (rsq < c.rc2) {
                double fpair, u = 0.0;
                pair_terms<MIXED, EV>(rsq, c, fpair, u);
                fx = fma(dx, fpair, fx);
                fy = fma(dy, fpair, fy);
                fz = fma(dz, fpair, fz);
                if (EV) {
                    const double hf = 0.5 * fpair;
                    acc[0] += 0.5 * u;
                    acc[1] = fma(dx * dx, hf, acc[1]);
                    acc[2] = fma(dy * dy, hf, acc[2]);
                    acc[3] = fma(dz * dz, hf, acc[3]);
                    acc[4] = fma(dx * dy, hf, acc[4]);
                    acc[5] = fma(dx * dz, hf, acc[5]);
                    acc[6] = fma(dy * dz, hf, acc[6]);
                }
            }
        }
        a.f[3 * i] = fx;
        a.f[3 * i + 1] = fy;
        a.f[3 * i + 2] = fz;
    }
    if (EV) block_partials<7>(acc, a.partials + blk * kPartVals);
}

template <int T, bool EV, bool MIXED>
__global__ __launch_bounds__(kThreads) void k_force_scatter(ForceArgs a, PairTab tab) {
    __shared__ CoefLds cl;
    if (T > 1) stage_coef(cl, tab);
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t i = blk * kThreads + threadIdx.x;
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    if (i < a.n) {
        const double xi = a.x[3 * i], yi = a.x[3 * i + 1], zi = a.x[3 * i + 2];
        const int ti = T > 1 ? a.type[i] : 0;
        const int nn = a.numneigh[i];
        const uint32_t *row = a.neigh + ((i >> 6) * (int64_t)a.cap) * kWave + (i & 63);
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int k = 0; k < nn; ++k) {
            const uint32_t raw = row[(int64_t)k * kWave];
            const int64_t j = raw & kIndexMask;
            double dx = xi - a.x[3 * j];
            double dy = yi - a.x[3 * j + 1];
            double dz = zi - a.x[3 * j + 2];
            const uint32_t code = raw >> kCodeShift;
            if (code) apply_image(code, a.box, dx, dy, dz);
            const double rsq = fma(dz, dz, fma(dy, dy, dx * dx));
            const int tj = T > 1 ? a.type[j] : 0;
            const Coef c = get_coef<T>(cl, tab, ti * T + tj);
            if (rsq < c.rc2) {
                double fpair, u = 0.0;
                pair_terms<MIXED, EV>(rsq, c, fpair, u);
                const double px = dx * fpair, py = dy * fpair, pz = dz * fpair;
                fx += px;
                fy += py;
                fz += pz;
                unsafeAtomicAdd(&a.f[3 * j], -px);
                unsafeAtomicAdd(&a.f[3 * j + 1], -py);
                unsafeAtomicAdd(&a.f[3 * j + 2], -pz);
                if (EV) {
                    acc[0] += u;
                    acc[1] = fma(dx * dx, fpair, acc[1]);
                    acc[2] = fma(dy * dy, fpair, acc[2]);
                    acc[3] = fma(dz * dz, fpair, acc[3]);
                    acc[4] = fma(dx * dy, fpair, acc[4]);
                    acc[5] = fma(dx * dz, fpair, acc[5]);
                    acc[6] = fma(dy * dz, fpair, acc[6]);
                }
            }
        }
        unsafeAtomicAdd(&a.f[3 * i], fx);
        unsafeAtomicAdd(&a.f[3 * i + 1], fy);
        unsafeAtomicAdd(&a.f[3 * i + 2], fz);
    }
    if (EV) block_partials<7>(acc, a.partials + blk * kPartVals);
}

// ---- batch of independent systems (global list format) ----
//
// One launch covers every system: atoms are numbered across the batch and
// each atom reads the box of its own system for the image codes.  LPA lanes
// share one atom's row (lane l takes entries l, l + LPA, ...; partial forces
// are summed across the LPA lanes in a fixed butterfly order), which keeps
// the lanes busy when systems are small; with `persistent` the grid is sized
// to the device and each workgroup strides over the atom groups.  Energy and
// virial, when requested, go to per-atom SoA arrays ev_atom[7][n] (half of
// every pair term), reduced per system afterwards.
struct BatchForceArgs {
    const double *x;
    const int32_t *type;
    int64_t n;
    const RepInfo *reps;
    const int32_t *rid;
    const int32_t *numneigh;
    const uint32_t *neigh;
    int cap;
    double *f;
    double *ev_atom;
};

// MULTI: more than one atom type (coefficients from LDS, indexed by the
// runtime type count).
template <bool MULTI, bool EV, bool MIXED, int LPA, int NT>
__global__ __launch_bounds__(NT) void k_force_batch(BatchForceArgs a, PairTab tab) {
    __shared__ CoefLds cl;
    if (MULTI) stage_coef(cl, tab);
    const int nt = tab.ntypes;
    constexpr int kPer = NT / LPA;  // atoms per workgroup pass
    const int sub = (int)(threadIdx.x % LPA);
    const int64_t grp = threadIdx.x / LPA;
    const int64_t passes = (a.n + kPer - 1) / kPer;
    for (int64_t p = xcd_remap(blockIdx.x, gridDim.x); p < passes; p += gridDim.x) {
        const int64_t i = p * kPer + grp;
        const bool active = i < a.n;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        double acc[7] = {0, 0, 0, 0, 0, 0, 0};
        if (active) {
            const Box box = a.reps[a.rid[i]].box;
            const double xi = a.x[3 * i], yi = a.x[3 * i + 1], zi = a.x[3 * i + 2];
            const int ti = MULTI ? a.type[i] : 0;
            const int nn = a.numneigh[i];
            const uint32_t *row = a.neigh + ((i >> 6) * (int64_t)a.cap) * kWave + (i & 63);
            for (int k = sub; k < nn; k += LPA) {
                const uint32_t raw = row[(int64_t)k * kWave];
                const int64_t j = raw & kIndexMask;
                double dx = xi - a.x[3 * j];
                double dy = yi - a.x[3 * j + 1];
                double dz = zi - a.x[3 * j + 2];
                const uint32_t code = raw >> kCodeShift;
                if (code) apply_image(code, box, dx, dy, dz);
                const double rsq = fma(dz, dz, fma(dy, dy, dx * dx));
                const int tj = MULTI ? a.type[j] : 0;
                const Coef c = get_coef<MULTI ? 2 : 1>(cl, tab, ti * nt + tj);
                if (rsq < c.rc2) {
                    double fpair, u = 0.0;
                    pair_terms<MIXED, EV>(rsq, c, fpair, u);
                    fx = fma(dx, fpair, fx);
                    fy = fma(dy, fpair, fy);
                    fz = fma(dz, fpair, fz);
                    if (EV) {
                        const double hf = 0.5 * fpair;
                        acc[0] += 0.5 * u;
                        acc[1] = fma(dx * dx, hf, acc[1]);
                        acc[2] = fma(dy * dy, hf, acc[2]);
                        acc[3] = fma(dz * dz, hf, acc[3]);
                        acc[4] = fma(dx * dy, hf, acc[4]);
                        acc[5] = fma(dx * dz, hf, acc[5]);
                        acc[6] = fma(dy * dz, hf, acc[6]);
                    }
                }
            }
        }
#pragma unroll
        for (int o = 1; o < LPA; o <<= 1) {
            fx += __shfl_xor(fx, o, kWave);
            fy += __shfl_xor(fy, o, kWave);
            fz += __shfl_xor(fz, o, kWave);
            if (EV) {
#pragma unroll
                for (int k = 0; k < 7; ++k) acc[k] += __shfl_xor(acc[k], o, kWave);
            }
        }
        if (active && sub == 0) {
            a.f[3 * i] = fx;
            a.f[3 * i + 1] = fy;
            a.f[3 * i + 2] = fz;
            if (EV) {
#pragma unroll
                for (int k = 0; k < 7; ++k) a.ev_atom[k * a.n + i] = acc[k];
            }
        }
    }
}

template <bool MULTI, bool EV, bool MIXED>
hipError_t launch_batch3(const BatchForceArgs &a, const PairTab &tab, int lpa, int block,
                         int persistent, hipStream_t s) {
    int dev = 0, cus = 256;
    if (persistent) {
        if (hipGetDevice(&dev) == hipSuccess)
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    }
    auto go = [&](auto kern, int nt) {
        const int64_t per = nt / lpa;
        const int64_t passes = (a.n + per - 1) / per;
        int64_t grid = passes;
        if (persistent) grid = std::min<int64_t>(passes, (int64_t)cus * persistent);
        if (grid < 1) grid = 1;
        kern<<<(unsigned)grid, nt, 0, s>>>(a, tab);
    };
#define LJMD_BATCH_CASE(L, B)                                      \
    if (lpa == L && block == B) {                                  \
        go(k_force_batch<MULTI, EV, MIXED, L, B>, B);              \
        return hipGetLastError();                                  \
    }
    LJMD_BATCH_CASE(1, 128)
    LJMD_BATCH_CASE(1, 256)
    LJMD_BATCH_CASE(2, 128)
    LJMD_BATCH_CASE(2, 256)
    LJMD_BATCH_CASE(4, 128)
    LJMD_BATCH_CASE(4, 256)
#undef LJMD_BATCH_CASE
    return hipErrorInvalidValue;
}

template <bool MULTI>
hipError_t launch_batch2(const BatchForceArgs &a, const PairTab &tab, int mixed, int ev, int lpa,
                         int block, int persistent, hipStream_t s) {
    if (ev)
        return mixed ? launch_batch3<MULTI, true, true>(a, tab, lpa, block, persistent, s)
                     : launch_batch3<MULTI, true, false>(a, tab, lpa, block, persistent, s);
    return mixed ? launch_batch3<MULTI, false, true>(a, tab, lpa, block, persistent, s)
                 : launch_batch3<MULTI, false, false>(a, tab, lpa, block, persistent, s);
}

// ---- tiled list: neighbor positions staged in LDS ----
//
// One workgroup per tile (tile.hpp).  The tile's stencil atoms are staged
// into LDS with their periodic shift added, so that x_i - staged_j is the
// minimum-image displacement.  When the whole stencil fits (the usual case)
// it is staged once and each lane walks its row word by word: four 16-bit
// slots per 64-bit word, unrolled with constant shifts, the cutoff applied
// by a select, and the row's words loaded four words ahead.  A stencil that
// does not fit is processed in chunks, each lane consuming the entries of its
// (increasing) row that fall into the current chunk.

constexpr int kGatherK = 2560;      // staged slots held at once by the gather
constexpr int kWaitVmcnt0 = 0x0F70;  // s_waitcnt vmcnt(0) expcnt(7) lgkmcnt(15) (gfx9 encoding)
constexpr int kScatterChunk = 1024; // positions + force accumulators (48 KB)

struct TileForceArgs {
    TileArgs t;
    const double *x;
    const int32_t *type;
    const int32_t *numneigh;
    const uint64_t *words;
    int capw;
    int sorted;
    double *f;
    double *partials;
    Kick kick;  // fused velocity-Verlet update (gather only; mode 0: none)
    FmOut fm;   // fused force-matching gradient (gather only; g null: none)
    // gather with energy/virial in a batch: each atom's half of its pair
    // terms, ev_atom[k * n + atom] (E, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz); else null
    double *ev_atom;
    int64_t n;
    int64_t ntiles;  // tiles of the list (the grid may be smaller: tile_walk)
};

// a[t] for a per-lane t, with uniform loads and selects only.
__device__ __forceinline__ double sel_type(const double (&a)[kMaxTypes], int t) {
    double r = a[0];
    r = t == 1 ? a[1] : r;
    r = t == 2 ? a[2] : r;
    r = t == 3 ? a[3] : r;
    return r;
}

// Row cursor over packed 16-bit slots, one 64-bit word (4 entries) ahead.
// It visits the words first, first + stride, first + 2 stride, ... of the
// row (stride > 1 when several lanes share one row); k is the row-wide index
// of the current entry and nn the row's entry count.
struct RowCursor {
    const uint64_t *words;
    int64_t s;
    int capw, nn, k, stride;
    uint64_t cur, next;
    __device__ __forceinline__ void init(const uint64_t *w, int64_t s_, int capw_, int nn_,
                                         int first = 0, int stride_ = 1) {
        words = w;
        s = s_;
        capw = capw_;
        nn = nn_;
        stride = stride_;
        k = 4 * first;
        cur = k < nn ? w[tile_word(s, first, capw)] : 0;
        next = k + 4 * stride < nn ? w[tile_word(s, first + stride, capw)] : 0;
    }
    __device__ __forceinline__ int32_t slot() const {
        return (int32_t)((cur >> (16 * (k & 3))) & 0xFFFFu);
    }
    __device__ __forceinline__ void advance() {
        ++k;
        if ((k & 3) == 0) {
            k += 4 * (stride - 1);
            cur = next;
            const int wn = (k >> 2) + stride;
            if (4 * wn < nn) next = words[tile_word(s, wn, capw)];
        }
    }
};

// The four entries of one list word (rows are padded with the null slot,
// which lies outside every cutoff, so no entry needs masking), written stage
// by stage across the four so that their LDS reads are issued together and
// their dependency chains interleave.
template <int T, bool EV, bool MIXED, bool WIN = false>
__device__ __forceinline__ void gather_word(uint64_t w, int32_t lo, int32_t hi, double xi,
                                            double yi, double zi, int ti,
                                            const double2 *sxy, const double *sz,
                                            const uint8_t *st,
                                            const CoefLds &cl, const PairTab &tab, double &fx,
                                            double &fy, double &fz, double (&acc)[7]) {
    int32_t m[4];
    m[0] = (int32_t)(w & 0xFFFFu);
    m[1] = (int32_t)((w >> 16) & 0xFFFFu);
    m[2] = (int32_t)((w >> 32) & 0xFFFFu);
    m[3] = (int32_t)(w >> 48);
    if (WIN) {
        // staged slots [lo, hi) only; every other entry reads the null slot
#pragma unroll
        for (int i = 0; i < 4; ++i) m[i] = (m[i] >= lo && m[i] < hi) ? m[i] - lo : hi - lo;
    }
    double dx[4], dy[4], dz[4], rsq[4];
    Coef c[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double2 pxy = sxy[m[i]];
        dx[i] = xi - pxy.x;
        dy[i] = yi - pxy.y;
        dz[i] = zi - sz[m[i]];
        c[i] = get_coef<T>(cl, tab, ti * T + (T > 1 ? (int)st[m[i]] : 0));
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) rsq[i] = fma(dz[i], dz[i], fma(dy[i], dy[i], dx[i] * dx[i]));
    double fpair[4], ue[4];
    if (MIXED) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float r2i = __builtin_amdgcn_rcpf((float)rsq[i]);
            r2i = rsq[i] < c[i].rc2 ? r2i : 0.0f;
            const float r6i = r2i * r2i * r2i;
            fpair[i] = (double)(r6i * (c[i].lj1f * r6i - c[i].lj2f) * r2i);
            if (EV) ue[i] = (double)(r6i * (c[i].lj3f * r6i - c[i].lj4f));
        }
    } else {
        double r2i[4];
        recip2(rsq[0], rsq[1], r2i[0], r2i[1]);
        recip2(rsq[2], rsq[3], r2i[2], r2i[3]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double q = cut_r2i(r2i[i], rsq[i] < c[i].rc2);
            const double r6i = q * q * q;
            fpair[i] = r6i * fma(c[i].lj1, r6i, -c[i].lj2) * q;
            if (EV) ue[i] = r6i * fma(c[i].lj3, r6i, -c[i].lj4);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        fx = fma(dx[i], fpair[i], fx);
        fy = fma(dy[i], fpair[i], fy);
        fz = fma(dz[i], fpair[i], fz);
        if (EV) {
            const double hf = 0.5 * fpair[i];
            acc[0] = fma(0.5, ue[i], acc[0]);
            acc[1] = fma(dx[i] * dx[i], hf, acc[1]);
            acc[2] = fma(dy[i] * dy[i], hf, acc[2]);
            acc[3] = fma(dz[i] * dz[i], hf, acc[3]);
            acc[4] = fma(dx[i] * dy[i], hf, acc[4]);
            acc[5] = fma(dx[i] * dz[i], hf, acc[5]);
            acc[6] = fma(dy[i] * dz[i], hf, acc[6]);
        }
    }
}

// Block-wide fixed-order sum of the per-lane energy/virial accumulators
// (slots 0-6) and kinetic energy (slot 7).
__device__ __forceinline__ void tile_partials(double (&v)[7], double ke, double *out) {
    __shared__ double s[kTileThreads / kWave][8];
#pragma unroll
    for (int k = 0; k < 7; ++k) v[k] = wave_sum(v[k]);
    ke = wave_sum(ke);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 7; ++k) s[threadIdx.x >> 6][k] = v[k];
        s[threadIdx.x >> 6][7] = ke;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double t = 0.0;
        for (int w = 0; w < kTileThreads / kWave; ++w) t += s[w][threadIdx.x];
        out[threadIdx.x] = t;
    }
}

// Full list.  LPA lanes share one home atom: lane `sub` of an atom takes the
// words sub, sub + LPA, ... of its (padded) row, and the partial forces are
// summed across the LPA lanes at the end in a fixed butterfly order.  Sharing
// a row evens out the per-wave work: a wave runs as long as its longest row,
// and with LPA = 4 a wave spans 16 rows instead of 64 (the lanes keep the
// rows' cell order, which is what makes the list-word loads of a wave
// contiguous).  `whole`: the stencil and its null slot
// have been staged by the caller; otherwise the stencil is staged here in
// chunks.  Adds this lane's energy/virial and kinetic energy to acc and ke.
template <int T, bool EV, bool MIXED, int LPA>
__device__ __forceinline__ void gather_rows(const TileForceArgs &a, const PairTab &tab,
                                            const TileArgs &ta, const TileGeom &tg,
                                            const TileLds &L, const RowTab &R,
                                            const CoefLds &cl, double2 *s_xy, double *s_z,
                                            uint8_t *s_t, int32_t h_lo, int32_t nh,
                                            int32_t total, bool whole,
                                            double fmw, double (&acc)[7], double &ke) {
    static_assert(LPA == 1 || LPA == 2 || LPA == 4 || LPA == 8, "lanes per atom");
    constexpr int kAtoms = kTileThreads / LPA;  // home atoms per pass
    constexpr int S = LPA == 1 ? kRowPad / 4 : 1;  // words per register set
    const int sub = (int)(threadIdx.x % LPA);
    for (int32_t h0 = h_lo; h0 < nh; h0 += kAtoms) {
        const int32_t h = h0 + (int32_t)(threadIdx.x / LPA);
        const bool active = h < nh;
        int32_t s = 0;
        int64_t u = 0;
        double xi = 0.0, yi = 0.0, zi = 0.0;
        int ti = 0, nn = 0;
        if (active) {
            s = tile_home_s(L, tg, h);
            u = a.sorted ? s : ta.perm[s];
            xi = a.x[3 * u];
            yi = a.x[3 * u + 1];
            zi = a.x[3 * u + 2];
            if (T > 1) ti = a.type[u];
            nn = a.numneigh[s];
        }
        double fx = 0.0, fy = 0.0, fz = 0.0;
        double racc[7] = {0, 0, 0, 0, 0, 0, 0};  // this row's energy/virial
        if (whole) {
            // This lane's words (padded to whole register sets) are software-
            // pipelined in two register sets of S words (a: words w .. w+S-1,
            // b: w+S .. w+2S-1 of the lane's sequence): each set is reloaded
            // right after it has been consumed, so its loads are in flight
            // while the other set is computed, and the reload can take the
            // registers of the consumed words (no copies, hence no early
            // waits).  Loads are unconditional, their index clamped to the
            // lane's last word; the words read past it are never consumed.
            // Inactive lanes read row 0 and never enter the loop.
            // this lane's words, a multiple of S
            const int nwl = (tile_row_words(nn) - sub + LPA - 1) / LPA;
            const int last = nwl > 0 ? nwl - 1 : 0;
            const uint64_t *wp =
                a.words + ((int64_t)(s >> 6) * a.capw + sub) * kWave + (s & 63);
            constexpr int64_t kStep = (int64_t)LPA * kWave;  // one word of this lane
            uint64_t p[2 * S];
#pragma unroll
            for (int k = 0; k < 2 * S; ++k) p[k] = wp[(int64_t)min(k, last) * kStep];
            // (the selects keep the compiler from turning a loop-carried
            // word into a load at the top of the loop; the first one's
            // condition is one the loop guard does not imply, so that it is
            // not folded away)
            uint64_t wa[S], wb[S];
            wa[0] = total > 0 ? p[0] : 0;
#pragma unroll
            for (int k = 1; k < S; ++k) wa[k] = nwl > k ? p[k] : 0;
#pragma unroll
            for (int k = 0; k < S; ++k) wb[k] = nwl > S + k ? p[S + k] : 0;
            // Wait here for the first words (needed right away anyway), so
            // that no load of the set-up is pending at the loop entry and the
            // waits inside the loop count only the loop's own loads.
            __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
            for (int w = 0; w < nwl; w += 2 * S) {
#pragma unroll
                for (int k = 0; k < S; ++k)
                    gather_word<T, EV, MIXED>(wa[k], 0, 0, xi, yi, zi, ti, s_xy, s_z, s_t, cl, tab,
                                              fx, fy, fz, racc);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k = 0; k < S; ++k) wa[k] = wp[(int64_t)min(w + 2 * S + k, last) * kStep];
                if (w + S < nwl) {
#pragma unroll
                    for (int k = 0; k < S; ++k)
                        gather_word<T, EV, MIXED>(wb[k], 0, 0, xi, yi, zi, ti, s_xy, s_z, s_t, cl,
                                                  tab, fx, fy, fz, racc);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k = 0; k < S; ++k) wb[k] = wp[(int64_t)min(w + 3 * S + k, last) * kStep];
            }
        } else {
            // stencil chunks of kGatherK - 1 slots, each staged with the null
            // slot after it; the lane keeps a cursor into its words (entries
            // ascend within a word: entry 0 is its smallest slot, entry 3 its
            // largest), uses a word in every chunk its entries fall in
            // (entries of other chunks read the null slot) and reads no word
            // in a chunk that holds none of its entries
            constexpr int32_t pay = kGatherK - 1;
            const int nw = tile_row_words(nn);
            const uint64_t *wp = a.words + (int64_t)(s >> 6) * a.capw * kWave + (s & 63);
            int w = sub;
            uint64_t cur = w < nw ? wp[(int64_t)w * kWave] : 0;
            for (int32_t lo = 0; lo < total; lo += pay) {
                const int32_t hi = min(total, lo + pay);
                __syncthreads();
                tile_stage<T, 0, false, true>(ta, tg, R, lo, hi, a.sorted, a.x, a.type, nullptr,
                                              s_xy, s_z, s_t, nullptr, nullptr, nullptr);
                if (threadIdx.x == 0) {
                    s_xy[hi - lo] = make_double2(kNullCoord, kNullCoord);
                    s_z[hi - lo] = kNullCoord;
                    if (T > 1) s_t[hi - lo] = 0;
                }
                __syncthreads();
                while (w < nw && (int32_t)(cur & 0xFFFFu) < hi) {
                    const uint64_t nxt = w + LPA < nw ? wp[(int64_t)(w + LPA) * kWave] : 0;
                    gather_word<T, EV, MIXED, true>(cur, lo, hi, xi, yi, zi, ti, s_xy, s_z, s_t,
                                                    cl, tab, fx, fy, fz, racc);
                    if ((int32_t)(cur >> 48) >= hi) break;  // continues in a later chunk
                    cur = nxt;
                    w += LPA;
                }
            }
        }
        if (EV) {
#pragma unroll
            for (int k = 0; k < 7; ++k) acc[k] += racc[k];
        }
#pragma unroll
        for (int o = 1; o < LPA; o <<= 1) {
            fx += __shfl_xor(fx, o, kWave);
            fy += __shfl_xor(fy, o, kWave);
            fz += __shfl_xor(fz, o, kWave);
            if (EV && a.ev_atom) {
#pragma unroll
                for (int k = 0; k < 7; ++k) racc[k] += __shfl_xor(racc[k], o, kWave);
            }
        }
        if (EV && a.ev_atom && active && sub == 0) {
#pragma unroll
            for (int k = 0; k < 7; ++k) a.ev_atom[k * a.n + u] = racc[k];
        }
        bool bad = false;
        if (active && sub == 0) {
            if (a.f) {
                a.f[3 * u] = fx;
                a.f[3 * u + 1] = fy;
                a.f[3 * u + 2] = fz;
            }
            if (a.fm.g) {
                a.fm.g[3 * u] = (fx - a.fm.ft[3 * u]) * fmw;
                a.fm.g[3 * u + 1] = (fy - a.fm.ft[3 * u + 1]) * fmw;
                a.fm.g[3 * u + 2] = (fz - a.fm.ft[3 * u + 2]) * fmw;
            }
            if (a.kick.mode) {
                // the same fmas as the separate kick kernels, so the
                // trajectory is bit-identical to running them apart
                const Kick &k = a.kick;
                const double hk = T > 1 ? sel_type(k.h, ti) : k.h[0];
                double vx = fma(hk, fx, k.v[3 * u]);
                double vy = fma(hk, fy, k.v[3 * u + 1]);
                double vz = fma(hk, fz, k.v[3 * u + 2]);
                bad = !(isfinite(vx) && isfinite(vy) && isfinite(vz));
                if (EV) {
                    const double m = T > 1 ? sel_type(k.mass, ti) : k.mass[0];
                    ke += 0.5 * m * vx * vx;
                    ke += 0.5 * m * vy * vy;
                    ke += 0.5 * m * vz * vz;
                }
                if (k.mode == 2) {
                    vx = fma(hk, fx, vx);
                    vy = fma(hk, fy, vy);
                    vz = fma(hk, fz, vz);
                    k.xnext[3 * u] = fma(k.dt, vx, xi);
                    k.xnext[3 * u + 1] = fma(k.dt, vy, yi);
                    k.xnext[3 * u + 2] = fma(k.dt, vz, zi);
                }
                k.v[3 * u] = vx;
                k.v[3 * u + 1] = vy;
                k.v[3 * u + 2] = vz;
            }
        }
        if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&a.kick.status[3], 1);
    }
}

// LPA lanes per home atom, or with LPA = 0 the lanes chosen per tile from
// its home count (tiles of a batch differ widely in size).  One workgroup per
// tile, or with WALK a smaller grid whose workgroups walk the tiles
// (tile_walk); the walking loop is a separate instantiation because keeping
// the tile's set-up live across iterations costs registers.  At least 4 waves
// per SIMD (two workgroups per compute unit, as the LDS stage allows).
template <int T, bool EV, bool MIXED, int LPA, bool WALK>
__global__ __launch_bounds__(kTileThreads, 4) void k_force_tile_gather(TileForceArgs a, PairTab tab) {
    static_assert(LPA == 0 || LPA == 1 || LPA == 2 || LPA == 4 || LPA == 8, "lanes per atom");
    __shared__ TileLds L;
    __shared__ RowTab R;
    __shared__ double2 s_xy[kGatherK];
    __shared__ double s_z[kGatherK];
    __shared__ uint8_t s_t[T > 1 ? kGatherK : 1];
    __shared__ CoefLds cl;
    if (T > 1) stage_coef(cl, tab);
    auto tile = [&](int64_t lb) {
        // The set-up and the staging are chains of memory round trips with
        // few instructions; while they run, their waves' instructions go
        // before those of the other workgroup's rows on the compute unit
        // (one workgroup per tile; the walking grid keeps one priority).
        if constexpr (!WALK) __builtin_amdgcn_s_setprio(1);
        int64_t lbl = 0;
        const TileArgs ta = tile_args_of(a.t, lb, lbl);
        const TileGeom tg = tile_setup(ta, lbl, L, &R);
        const int32_t total = L.off[tg.ncells];
        const int32_t nh = tile_home_count(L, tg);
        const bool whole = total < kGatherK;  // the stencil and the null slot fit
        // force-matching weight of the tile's system
        double fmw = 0.0;
        if (a.fm.g) {
            const int64_t r = a.t.reps ? (int64_t)a.t.tile_rep[lb] : 0;
            fmw = a.fm.wsys ? a.fm.wsys[r]
                            : 2.0 / (double)(a.t.reps ? a.t.reps[r].natoms : a.n);
        }
        if (whole) {
            tile_stage<T, 0, false, true>(ta, tg, R, 0, total, a.sorted, a.x, a.type, nullptr, s_xy,
                                          s_z, s_t, nullptr, nullptr, nullptr);
            if (threadIdx.x == 0) {
                s_xy[total] = make_double2(kNullCoord, kNullCoord);
                s_z[total] = kNullCoord;
                if (T > 1) s_t[total] = 0;
            }
            __syncthreads();
        }
        if constexpr (!WALK) __builtin_amdgcn_s_setprio(0);
        double acc[7] = {0, 0, 0, 0, 0, 0, 0};  // block energy/virial, this lane's share
        double ke = 0.0;
        // home atoms [h_lo, h_hi) with `lanes` lanes per atom
        auto rows = [&](int lanes, int32_t h_lo, int32_t h_hi) {
            if (lanes == 8)
                gather_rows<T, EV, MIXED, 8>(a, tab, ta, tg, L, R, cl, s_xy, s_z, s_t, h_lo, h_hi,
                                             total, whole, fmw, acc, ke);
            else if (lanes == 4)
                gather_rows<T, EV, MIXED, 4>(a, tab, ta, tg, L, R, cl, s_xy, s_z, s_t, h_lo, h_hi,
                                             total, whole, fmw, acc, ke);
            else if (lanes == 2)
                gather_rows<T, EV, MIXED, 2>(a, tab, ta, tg, L, R, cl, s_xy, s_z, s_t, h_lo, h_hi,
                                             total, whole, fmw, acc, ke);
            else
                gather_rows<T, EV, MIXED, 1>(a, tab, ta, tg, L, R, cl, s_xy, s_z, s_t, h_lo, h_hi,
                                             total, whole, fmw, acc, ke);
        };
        if constexpr (LPA == 0 || LPA == 1) {
            // whole passes of one lane per atom, then the remaining atoms of a
            // tile with more home atoms than lanes with as many lanes per atom
            // as cover them in one pass (a partly filled pass at one lane per
            // atom would take about as long as a full one)
            int32_t h = 0;
            if (LPA == 1 || tile_pass_lanes(nh) == 1) {
                h = nh - nh % kTileThreads;
                if (h > 0)
                    gather_rows<T, EV, MIXED, 1>(a, tab, ta, tg, L, R, cl, s_xy, s_z, s_t, 0, h,
                                                 total, whole, fmw, acc, ke);
            }
            if (h < nh) rows(tile_pass_lanes(nh - h), h, nh);
        } else {
            gather_rows<T, EV, MIXED, LPA>(a, tab, ta, tg, L, R, cl, s_xy, s_z, s_t, 0, nh, total,
                                           whole, fmw, acc, ke);
        }
        if (EV) tile_partials(acc, ke, a.partials + lb * kPartVals);
    };
    if constexpr (WALK) {
        const TileWalk tw = tile_walk(a.ntiles);
        for (int64_t lb = tw.first; lb < tw.end; lb += tw.step) {
            if (lb != tw.first) __syncthreads();  // the previous tile is done with the LDS
            tile(lb);
        }
    } else {
        tile(xcd_remap(blockIdx.x, gridDim.x));
    }
}

// Half list: the partner's share is accumulated in LDS per staged slot and
// added to global memory once per chunk (FP64 atomics), the atom's own share
// once at the end.
template <int T, bool EV, bool MIXED>
__global__ __launch_bounds__(kTileThreads) void k_force_tile_scatter(TileForceArgs a,
                                                                    PairTab tab) {
    __shared__ TileLds L;
    __shared__ RowTab R;
    __shared__ double2 s_xy[kScatterChunk];
    __shared__ double s_z[kScatterChunk];
    __shared__ double s_fx[kScatterChunk], s_fy[kScatterChunk], s_fz[kScatterChunk];
    __shared__ uint32_t s_u[kScatterChunk];
    __shared__ uint8_t s_t[T > 1 ? kScatterChunk : 1];
    __shared__ CoefLds cl;
    if (T > 1) stage_coef(cl, tab);
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    int64_t lbl = 0;
    const TileArgs ta = tile_args_of(a.t, lb, lbl);
    const TileGeom tg = tile_setup(ta, lbl, L, &R);
    const int32_t total = L.off[tg.ncells];
    const int32_t nh = tile_home_count(L, tg);
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int32_t h0 = 0; h0 < nh; h0 += kTileThreads) {
        const int32_t h = h0 + (int32_t)threadIdx.x;
        const bool active = h < nh;
        int32_t s = 0;
        int64_t u = 0;
        double xi = 0.0, yi = 0.0, zi = 0.0;
        int ti = 0;
        RowCursor rc;
        rc.init(a.words, 0, a.capw, 0);
        if (active) {
            s = tile_home_s(L, tg, h);
            u = a.sorted ? s : ta.perm[s];
            xi = a.x[3 * u];
            yi = a.x[3 * u + 1];
            zi = a.x[3 * u + 2];
            if (T > 1) ti = a.type[u];
            rc.init(a.words, s, a.capw, a.numneigh[s]);
        }
        double fx = 0.0, fy = 0.0, fz = 0.0;
        // every partner of a tiled half list follows its home atom in the
        // stage (forward half stencil), so the slots before the first home
        // cell are neither read nor updated
        const int32_t first = L.off[(tg.b[1] + 3) * tg.w + 1];
        for (int32_t lo = first; lo < total; lo += kScatterChunk) {
            const int32_t hi = min(total, lo + kScatterChunk);
            __syncthreads();
            tile_stage<T, 1, false, true>(ta, tg, R, lo, hi, a.sorted, a.x, a.type, nullptr, s_xy,
                                          s_z, s_t, s_u, nullptr, nullptr);
            for (int32_t q = (int32_t)threadIdx.x; q < hi - lo; q += kTileThreads)
                s_fx[q] = s_fy[q] = s_fz[q] = 0.0;
            __syncthreads();
            while (rc.k < rc.nn) {
                const int32_t q = rc.slot();
                if (q >= hi) break;
                const int32_t m = q - lo;
                const double2 pxy = s_xy[m];
                const double dx = xi - pxy.x;
                const double dy = yi - pxy.y;
                const double dz = zi - s_z[m];
                const double rsq = fma(dz, dz, fma(dy, dy, dx * dx));
                const Coef c = get_coef<T>(cl, tab, ti * T + (T > 1 ? (int)s_t[m] : 0));
                if (rsq < c.rc2) {
                    double fpair, ue = 0.0;
                    pair_terms<MIXED, EV>(rsq, c, fpair, ue);
                    const double px = dx * fpair, py = dy * fpair, pz = dz * fpair;
                    fx += px;
                    fy += py;
                    fz += pz;
                    unsafeAtomicAdd(&s_fx[m], -px);
                    unsafeAtomicAdd(&s_fy[m], -py);
                    unsafeAtomicAdd(&s_fz[m], -pz);
                    if (EV) {
                        acc[0] += ue;
                        acc[1] = fma(dx * dx, fpair, acc[1]);
                        acc[2] = fma(dy * dy, fpair, acc[2]);
                        acc[3] = fma(dz * dz, fpair, acc[3]);
                        acc[4] = fma(dx * dy, fpair, acc[4]);
                        acc[5] = fma(dx * dz, fpair, acc[5]);
                        acc[6] = fma(dy * dz, fpair, acc[6]);
                    }
                }
                rc.advance();
            }
            __syncthreads();
            for (int32_t q = (int32_t)threadIdx.x; q < hi - lo; q += kTileThreads) {
                const double vx = s_fx[q], vy = s_fy[q], vz = s_fz[q];
                if (vx != 0.0 || vy != 0.0 || vz != 0.0) {
                    const int64_t uj = s_u[q];
                    unsafeAtomicAdd(&a.f[3 * uj], vx);
                    unsafeAtomicAdd(&a.f[3 * uj + 1], vy);
                    unsafeAtomicAdd(&a.f[3 * uj + 2], vz);
                }
            }
        }
        if (active) {
            unsafeAtomicAdd(&a.f[3 * u], fx);
            unsafeAtomicAdd(&a.f[3 * u + 1], fy);
            unsafeAtomicAdd(&a.f[3 * u + 2], fz);
        }
    }
    if (EV) tile_partials(acc, 0.0, a.partials + lb * kPartVals);
}

template <int T, bool EV, bool MIXED>
hipError_t launch_tile3(const TileForceArgs &a, const PairTab &tab, int half, int lpa,
                        unsigned blocks, hipStream_t s) {
    const bool walk = (int64_t)blocks < a.ntiles;  // a persistent grid (batch tuning)
    if (half)
        k_force_tile_scatter<T, EV, MIXED><<<blocks, kTileThreads, 0, s>>>(a, tab);
    else if (walk && lpa == 4)
        k_force_tile_gather<T, EV, MIXED, 4, true><<<blocks, kTileThreads, 0, s>>>(a, tab);
    else if (walk && lpa == 2)
        k_force_tile_gather<T, EV, MIXED, 2, true><<<blocks, kTileThreads, 0, s>>>(a, tab);
    else if (walk && lpa == 1)
        k_force_tile_gather<T, EV, MIXED, 1, true><<<blocks, kTileThreads, 0, s>>>(a, tab);
    else if (walk)
        k_force_tile_gather<T, EV, MIXED, 0, true><<<blocks, kTileThreads, 0, s>>>(a, tab);
    else if (lpa == 8)
        k_force_tile_gather<T, EV, MIXED, 8, false><<<blocks, kTileThreads, 0, s>>>(a, tab);
    else if (lpa == 4)
        k_force_tile_gather<T, EV, MIXED, 4, false><<<blocks, kTileThreads, 0, s>>>(a, tab);
    else if (lpa == 2)
        k_force_tile_gather<T, EV, MIXED, 2, false><<<blocks, kTileThreads, 0, s>>>(a, tab);
    else if (lpa == 1)
        k_force_tile_gather<T, EV, MIXED, 1, false><<<blocks, kTileThreads, 0, s>>>(a, tab);
    else
        k_force_tile_gather<T, EV, MIXED, 0, false><<<blocks, kTileThreads, 0, s>>>(a, tab);
    return hipGetLastError();
}

template <int T>
hipError_t launch_tile2(const TileForceArgs &a, const PairTab &tab, int half, int mixed, int ev,
                        int lpa, unsigned blocks, hipStream_t s) {
    if (ev) {
        return mixed ? launch_tile3<T, true, true>(a, tab, half, lpa, blocks, s)
                     : launch_tile3<T, true, false>(a, tab, half, lpa, blocks, s);
    }
    return mixed ? launch_tile3<T, false, true>(a, tab, half, lpa, blocks, s)
                 : launch_tile3<T, false, false>(a, tab, half, lpa, blocks, s);
}

// Fixed-order sum of nblocks rows of partials: out[v] = sum_b p[b][v].
__global__ __launch_bounds__(kThreads) void k_reduce_partials(const double *__restrict__ p,
                                                              int64_t nblocks, int nvals,
                                                              double *__restrict__ out) {
    __shared__ double s[kThreads];
    for (int v = 0; v < nvals; ++v) {
        double t = 0.0;
        for (int64_t b = threadIdx.x; b < nblocks; b += kThreads) t += p[b * kPartVals + v];
        s[threadIdx.x] = t;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[v] = s[0];
        __syncthreads();
    }
}

template <int T, bool EV, bool MIXED>
hipError_t launch3(const ForceArgs &a, const PairTab &tab, int half, unsigned blocks,
                   hipStream_t s) {
    if (half)
        k_force_scatter<T, EV, MIXED><<<blocks, kThreads, 0, s>>>(a, tab);
    else
        k_force_gather<T, EV, MIXED><<<blocks, kThreads, 0, s>>>(a, tab);
    return hipGetLastError();
}

template <int T>
hipError_t launch2(const ForceArgs &a, const PairTab &tab, int half, int mixed, int ev,
                   unsigned blocks, hipStream_t s) {
    if (ev) {
        return mixed ? launch3<T, true, true>(a, tab, half, blocks, s)
                     : launch3<T, true, false>(a, tab, half, blocks, s);
    }
    return mixed ? launch3<T, false, true>(a, tab, half, blocks, s)
                 : launch3<T, false, false>(a, tab, half, blocks, s);
}

}  // namespace

hipError_t launch_forces(const double *x, const int32_t *type, int64_t n, const Box &box,
                         const PairTab &tab, const int32_t *numneigh, const uint32_t *neigh,
                         int cap, int half, int mixed, int ev, double *f, double *partials,
                         int64_t *nblocks_out, hipStream_t s) {
    const int64_t blocks = (n + kThreads - 1) / kThreads;
    *nblocks_out = blocks;
    if (n <= 0) return hipSuccess;
    if (half) {
        hipError_t e = launch_zero_f64(f, 3 * n, s);
        if (e != hipSuccess) return e;
    }
    ForceArgs a{x, type, n, box, numneigh, neigh, cap, f, partials};
    switch (tab.ntypes) {
        case 1: return launch2<1>(a, tab, half, mixed, ev, (unsigned)blocks, s);
        case 2: return launch2<2>(a, tab, half, mixed, ev, (unsigned)blocks, s);
        case 3: return launch2<3>(a, tab, half, mixed, ev, (unsigned)blocks, s);
        default: return launch2<4>(a, tab, half, mixed, ev, (unsigned)blocks, s);
    }
}

hipError_t launch_forces_tiled(const TileArgs &t, const double *x, const int32_t *type,
                               int64_t n, const PairTab &tab, const int32_t *numneigh,
                               const void *neigh, int cap, int sorted, int half, int mixed, int ev,
                               int lpa, double *f, double *partials, int64_t *nblocks_out,
                               hipStream_t s, const Kick *kick, double *ev_atom, int persistent,
                               const FmOut *fm) {
    const int64_t blocks = tile_blocks(t);
    *nblocks_out = blocks;
    // the full-list gather with persistent > 0: a grid of persistent x (compute
    // units) workgroups walking the tiles (never more workgroups than tiles)
    int64_t grid = blocks;
    if (persistent > 0 && !half && lpa != 8) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        grid = std::min<int64_t>(blocks, (int64_t)cus * persistent);
    }
    if (n <= 0) {
        *nblocks_out = 0;
        return hipSuccess;
    }
    if (half) {
        hipError_t e = launch_zero_f64(f, 3 * n, s);
        if (e != hipSuccess) return e;
    }
    TileForceArgs a{t, x, type, numneigh, static_cast<const uint64_t *>(neigh), tile_capw(cap),
                    sorted, f, partials, Kick{}, FmOut{nullptr, nullptr, nullptr}, ev_atom, n,
                    blocks};
    if (kick || fm) {
        if (half) return hipErrorInvalidValue;  // a scatter's forces are complete only at the end
        if (kick) a.kick = *kick;
        if (fm) a.fm = *fm;
    }
    if (!f && !a.fm.g) return hipErrorInvalidValue;
    switch (tab.ntypes) {
        case 1: return launch_tile2<1>(a, tab, half, mixed, ev, lpa, (unsigned)grid, s);
        case 2: return launch_tile2<2>(a, tab, half, mixed, ev, lpa, (unsigned)grid, s);
        case 3: return launch_tile2<3>(a, tab, half, mixed, ev, lpa, (unsigned)grid, s);
        default: return launch_tile2<4>(a, tab, half, mixed, ev, lpa, (unsigned)grid, s);
    }
}

hipError_t launch_forces_batch(const double *x, const int32_t *type, int64_t n,
                               const BatchView &b, const PairTab &tab, const int32_t *numneigh,
                               const uint32_t *neigh, int cap, int mixed, double *f,
                               double *ev_atom, int lanes_per_atom, int block, int persistent,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    BatchForceArgs a{x, type, n, b.reps, b.rid, numneigh, neigh, cap, f, ev_atom};
    const int ev = ev_atom != nullptr;
    if (tab.ntypes > 1)
        return launch_batch2<true>(a, tab, mixed, ev, lanes_per_atom, block, persistent, s);
    return launch_batch2<false>(a, tab, mixed, ev, lanes_per_atom, block, persistent, s);
}

// g = w (F - Ft) per atom (the force-matching gradient after a force kernel
// that cannot apply it itself), w of the atom's system as in FmOut.
__global__ __launch_bounds__(256) void k_fm_grad(const double *__restrict__ f, FmOut fm, int64_t n,
                                                 const RepInfo *__restrict__ reps,
                                                 const int32_t *__restrict__ rid) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t r = reps ? (int64_t)rid[i] : 0;
    const double w = fm.wsys ? fm.wsys[r] : 2.0 / (double)(reps ? reps[r].natoms : n);
#pragma unroll
    for (int d = 0; d < 3; ++d) fm.g[3 * i + d] = (f[3 * i + d] - fm.ft[3 * i + d]) * w;
}

hipError_t launch_fm_grad(const double *f, const FmOut &fm, int64_t n, const RepInfo *reps,
                          const int32_t *rid, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fm_grad<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(f, fm, n, reps, rid);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const double *partials, int64_t nblocks, int nvals,
                                  double *out, hipStream_t s) {
    k_reduce_partials<<<1, kThreads, 0, s>>>(partials, nblocks, nvals, out);
    return hipGetLastError();
}

}  // namespace ljmd
