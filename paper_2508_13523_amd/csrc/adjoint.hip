// Adjoint of the Lennard-Jones force map: given g_i = dL/dF_i, the gradient
// of a scalar loss L(F) with respect to positions and the eps/sigma tables.
//
// The pair (i, j) adds gamma(r) d to F_i and -gamma(r) d to F_j, with
// d = x_i - x_j and gamma = fpair = lj1 r^-14 - lj2 r^-8 (lj1 = 48 eps s^12,
// lj2 = 24 eps s^6; Sec. 4, Eq. (1) and its pairwise derivative).  Hence,
// with gd = g_i - g_j and gamma'(r)/r = r^-10 (-14 lj1 r^-6 + 8 lj2):
//   dL/dx_i = sum_j [ gamma gd + (gamma'/r) (d . gd) d ]      (= -(H g)_i)
// which a full list evaluates as a gather, like the force.  At fixed r the
// parameter derivatives are d gamma/d eps = gamma/eps and
// d gamma/d sigma = r^-2 r^-6 (12 lj1 r^-6 - 6 lj2) / sigma, and each full-
// list entry adds half of (d gamma/d theta)(d . gd) to entry [t_i][t_j].
// The cutoffs are held fixed.
#include "tile.hpp"

#include <algorithm>

namespace ljmd {

namespace {

constexpr int kThreads = 256;

struct BwdArgs {
    const double *x;
    const int32_t *type;
    int64_t n;
    Box box;
    const int32_t *numneigh;
    const uint32_t *neigh;
    int cap;
    const double *g;
    double *gx;
    double *partials;
    const RepInfo *reps;  // batch: box of each atom's system (else `box`)
    const int32_t *rid;
};

__device__ __forceinline__ double recip(double a) {
    double y = __builtin_amdgcn_rcp(a);
    double e = fma(-a, y, 1.0);
    y = fma(y, e, y);
    e = fma(-a, y, 1.0);
    return fma(y, e, y);
}

struct BwdLds {
    double rc2[kTab], lj1[kTab], lj2[kTab], ieps[kTab], isig[kTab];
};

template <int T>
__global__ __launch_bounds__(kThreads) void k_backward(BwdArgs a, PairTab tab) {
    __shared__ BwdLds c;
    __shared__ double s_red[kThreads / kWave][kPartVals];
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kTab; ++k) {
            c.rc2[k] = tab.rc2[k];
            c.lj1[k] = tab.lj1[k];
            c.lj2[k] = tab.lj2[k];
            c.ieps[k] = tab.eps[k] > 0.0 ? 1.0 / tab.eps[k] : 0.0;
            c.isig[k] = tab.sig[k] > 0.0 ? 1.0 / tab.sig[k] : 0.0;
        }
    }
    __syncthreads();
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t i = blk * kThreads + threadIdx.x;
    double pe[T], ps[T];
#pragma unroll
    for (int b = 0; b < T; ++b) pe[b] = ps[b] = 0.0;
    int ti = 0;
    if (i < a.n) {
        const double xi = a.x[3 * i], yi = a.x[3 * i + 1], zi = a.x[3 * i + 2];
        const double gxi = a.g[3 * i], gyi = a.g[3 * i + 1], gzi = a.g[3 * i + 2];
        ti = T > 1 ? a.type[i] : 0;
        const Box box = a.reps ? a.reps[a.rid[i]].box : a.box;
        const int nn = a.numneigh[i];
        const uint32_t *row = a.neigh + ((i >> 6) * (int64_t)a.cap) * kWave + (i & 63);
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int k = 0; k < nn; ++k) {
            const uint32_t raw = row[(int64_t)k * kWave];
            const int64_t j = raw & kIndexMask;
            double dx = xi - a.x[3 * j];
            double dy = yi - a.x[3 * j + 1];
            double dz = zi - a.x[3 * j + 2];
            const uint32_t code = raw >> kCodeShift;
            if (code) {
                if (code & 1u) dx -= box.L[0];
                else if (code & 2u) dx += box.L[0];
                if (code & 4u) dy -= box.L[1];
                else if (code & 8u) dy += box.L[1];
                if (code & 16u) dz -= box.L[2];
                else if (code & 32u) dz += box.L[2];
            }
            const double rsq = fma(dz, dz, fma(dy, dy, dx * dx));
            const int tj = T > 1 ? a.type[j] : 0;
            const int k2 = ti * T + tj;
            if (rsq < c.rc2[k2]) {
                const double lj1 = c.lj1[k2], lj2 = c.lj2[k2];
                const double gdx = gxi - a.g[3 * j];
                const double gdy = gyi - a.g[3 * j + 1];
                const double gdz = gzi - a.g[3 * j + 2];
                const double dot = fma(dz, gdz, fma(dy, gdy, dx * gdx));
                const double r2i = recip(rsq);
                const double r6i = r2i * r2i * r2i;
                const double gam = r6i * fma(lj1, r6i, -lj2) * r2i;
                const double dgr = r2i * r2i * r6i * fma(-14.0 * lj1, r6i, 8.0 * lj2);
                const double t = dgr * dot;
                ax = fma(t, dx, fma(gam, gdx, ax));
                ay = fma(t, dy, fma(gam, gdy, ay));
                az = fma(t, dz, fma(gam, gdz, az));
                const double de = 0.5 * gam * c.ieps[k2] * dot;
                const double ds = 0.5 * r6i * r2i * fma(12.0 * lj1, r6i, -6.0 * lj2) *
                                  c.isig[k2] * dot;
#pragma unroll
                for (int b = 0; b < T; ++b) {
                    if (tj == b) {
                        pe[b] += de;
                        ps[b] += ds;
                    }
                }
            }
        }
        a.gx[3 * i] = ax;
        a.gx[3 * i + 1] = ay;
        a.gx[3 * i + 2] = az;
    }
    // per-block partials of the 2 T^2 parameter gradients, fixed order
#pragma unroll
    for (int ta = 0; ta < T; ++ta) {
#pragma unroll
        for (int b = 0; b < T; ++b) {
            const double ve = wave_sum(ti == ta ? pe[b] : 0.0);
            const double vs = wave_sum(ti == ta ? ps[b] : 0.0);
            if ((threadIdx.x & 63) == 0) {
                s_red[threadIdx.x >> 6][(ta * T + b) * 2] = ve;
                s_red[threadIdx.x >> 6][(ta * T + b) * 2 + 1] = vs;
            }
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < 2 * T * T) {
        double t = 0.0;
        for (int w = 0; w < kThreads / kWave; ++w) t += s_red[w][threadIdx.x];
        a.partials[blk * kPartVals + threadIdx.x] = t;
    }
}

// Tiled list: positions (with their periodic shift) and upstream gradients of
// the tile's stencil atoms are staged in LDS chunk by chunk; each lane walks
// its row of increasing 16-bit slots.
// Stencil slots staged at once (positions, gradients: 48 bytes each; one of
// them holds the null slot).  Two workgroups still fit a compute unit;
// larger stencils are processed in chunks.
constexpr int kBwdChunk = 1472;

// One list word (four entries) of a home atom against the staged slots: no
// branches; entries outside the cutoff are zeroed through their reciprocal
// square distance, and the row padding reads the null slot (far from every
// atom, gradient zero).  With WIN only the slots [lo, hi) are staged, the
// null slot right after them, and entries of other chunks read it too.
//
// With A = r^-14 and B = r^-8, gamma = lj1 A - lj2 B and gamma'/r =
// r^-2 (8 lj2 B - 14 lj1 A).  The parameter terms of an entry, half of
// (gamma/eps)(d . gd) and of (12 lj1 A - 6 lj2 B)/sigma (d . gd), are linear
// in A (d . gd) and B (d . gd) with per-type-pair factors, so the row only
// sums those two by partner type and the factors are applied per row: sa[0],
// sb[0] sum over all partners, sa[b], sb[b] (b >= 1) over partners of type b.
template <int T, bool WIN>
__device__ __forceinline__ void bwd_word(uint64_t w, int32_t lo, int32_t hi, double xi, double yi,
                                         double zi, double gxi, double gyi, double gzi, int ti,
                                         const double2 *sxy, const double *sz,
                                         const double2 *sgxy, const double *sgz,
                                         const uint8_t *st, const BwdLds &c, double &ax,
                                         double &ay, double &az, double (&sa)[T],
                                         double (&sb)[T]) {
    // the word's two pairs of entries one after the other (one shared
    // reciprocal per pair): half the live registers of all four at once, so
    // that two 512-lane workgroups fit a compute unit
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
        const uint32_t pair = (uint32_t)(w >> (32 * h));
        double dx[2], dy[2], dz[2], gdx[2], gdy[2], gdz[2], rsq[2], r2i[2];
        int tj[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int32_t q = (int32_t)((pair >> (16 * i)) & 0xFFFFu);
            const int32_t m = WIN ? ((q >= lo && q < hi) ? q - lo : hi - lo) : q;
            const double2 pxy = sxy[m];
            const double2 gxy = sgxy[m];
            dx[i] = xi - pxy.x;
            dy[i] = yi - pxy.y;
            dz[i] = zi - sz[m];
            gdx[i] = gxi - gxy.x;
            gdy[i] = gyi - gxy.y;
            gdz[i] = gzi - sgz[m];
            tj[i] = T > 1 ? (int)st[m] : 0;
            rsq[i] = fma(dz[i], dz[i], fma(dy[i], dy[i], dx[i] * dx[i]));
        }
        recip2(rsq[0], rsq[1], r2i[0], r2i[1]);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int k2 = ti * T + tj[i];
            const double q = cut_r2i(r2i[i], rsq[i] < c.rc2[k2]);
            const double r6i = q * q * q;
            const double B = q * r6i;
            const double A = B * r6i;
            const double l1a = c.lj1[k2] * A, l2b = c.lj2[k2] * B;
            const double gam = l1a - l2b;
            const double dgr = q * fma(-14.0, l1a, 8.0 * l2b);
            const double dot = fma(dz[i], gdz[i], fma(dy[i], gdy[i], dx[i] * gdx[i]));
            const double t = dgr * dot;
            ax = fma(t, dx[i], fma(gam, gdx[i], ax));
            ay = fma(t, dy[i], fma(gam, gdy[i], ay));
            az = fma(t, dz[i], fma(gam, gdz[i], az));
            const double ad = A * dot, bd = B * dot;
            sa[0] += ad;
            sb[0] += bd;
            if (T == 2) {
                const double w1 = (double)tj[i];  // 0 or 1: adds ad exactly or nothing
                sa[T - 1] = fma(ad, w1, sa[T - 1]);
                sb[T - 1] = fma(bd, w1, sb[T - 1]);
            } else {
#pragma unroll
                for (int b = 1; b < T; ++b) {
                    sa[b] += tj[i] == b ? ad : 0.0;
                    sb[b] += tj[i] == b ? bd : 0.0;
                }
            }
        }
    }
}

struct BwdTileArgs {
    TileArgs t;
    const double *x;
    const int32_t *type;
    const int32_t *numneigh;
    const uint64_t *words;
    int capw;
    int sorted;
    const double *g;
    double *gx;
    double *partials;
};

// Staged stencil slots of one adjoint workgroup (positions, gradients,
// types); slot hi - lo of a chunk [lo, hi) is the null slot.
template <int T>
struct BwdStage {
    double2 xy[kBwdChunk], gxy[kBwdChunk];
    double z[kBwdChunk], gz[kBwdChunk];
    uint8_t t[T > 1 ? kBwdChunk : 1];
};

template <int T>
__device__ __forceinline__ void bwd_stage(const BwdTileArgs &a, const TileArgs &ta,
                                          const TileGeom &tg, const RowTab &R, int32_t lo,
                                          int32_t hi, BwdStage<T> &S) {
    tile_stage<T, 0, true, true>(ta, tg, R, lo, hi, a.sorted, a.x, a.type, a.g, S.xy, S.z, S.t,
                                 nullptr, S.gxy, S.gz);
    if (threadIdx.x == 0) {
        S.xy[hi - lo] = make_double2(kNullCoord, kNullCoord);
        S.z[hi - lo] = kNullCoord;
        S.gxy[hi - lo] = make_double2(0.0, 0.0);
        S.gz[hi - lo] = 0.0;
        if (T > 1) S.t[hi - lo] = 0;
    }
}

// The home atoms of one tile with LPA lanes per atom (lane `sub` walks the
// words sub, sub + LPA, ... of the row, which stay in increasing slot
// order); the partial gradients are summed over the LPA lanes in a fixed
// butterfly order, and each row's parameter sums (see bwd_word) are added
// to this lane's SA, SB by type pair [t_i][t_j].
// A stencil that fits one chunk has been staged by the caller.  Otherwise
// the stencil is staged in chunks of `pay` slots and each lane keeps a
// cursor into its words: a word is used in every chunk its entries fall in
// (entries of other chunks read the null slot) and no word is read in a
// chunk that holds none of its entries.
template <int T, int LPA>
__device__ __forceinline__ void bwd_rows(const BwdTileArgs &a, const TileArgs &ta,
                                         const TileGeom &tg, const TileLds &L, const RowTab &R,
                                         const BwdLds &c, BwdStage<T> &S, int32_t nh,
                                         int32_t total, int nchunk, int32_t pay,
                                         double (&SA)[T * T], double (&SB)[T * T]) {
    constexpr int kAtoms = kTileThreads / LPA;
    const int sub = (int)(threadIdx.x % LPA);
    const int capw = a.capw;
    double sa[T], sb[T];  // this home atom's row (see bwd_word)
    for (int32_t h0 = 0; h0 < nh; h0 += kAtoms) {
        int ti = 0;
#pragma unroll
        for (int b = 0; b < T; ++b) sa[b] = sb[b] = 0.0;
        const int32_t h = h0 + (int32_t)(threadIdx.x / LPA);
        const bool active = h < nh;
        int32_t s = 0;
        int64_t u = 0;
        int nn = 0;
        double xi = 0.0, yi = 0.0, zi = 0.0, gxi = 0.0, gyi = 0.0, gzi = 0.0;
        if (active) {
            s = tile_home_s(L, tg, h);
            u = a.sorted ? s : ta.perm[s];
            xi = a.x[3 * u];
            yi = a.x[3 * u + 1];
            zi = a.x[3 * u + 2];
            gxi = a.g[3 * u];
            gyi = a.g[3 * u + 1];
            gzi = a.g[3 * u + 2];
            ti = T > 1 ? a.type[u] : 0;
            nn = a.numneigh[s];
        }
        double ax = 0.0, ay = 0.0, az = 0.0;
        const int nw = tile_row_words(nn);
        if (nchunk == 1) {
            // the lane's words two ahead of their use
            uint64_t w0 = sub < nw ? a.words[tile_word(s, sub, capw)] : 0;
            uint64_t w1 = sub + LPA < nw ? a.words[tile_word(s, sub + LPA, capw)] : 0;
#pragma unroll 1
            for (int w = sub; w < nw; w += LPA) {
                const uint64_t wd = w0;
                w0 = w1;
                if (w + 2 * LPA < nw) w1 = a.words[tile_word(s, w + 2 * LPA, capw)];
                bwd_word<T, false>(wd, 0, total, xi, yi, zi, gxi, gyi, gzi, ti, S.xy, S.z, S.gxy,
                                   S.gz, S.t, c, ax, ay, az, sa, sb);
            }
        } else {
            int w = sub;
            uint64_t cur = w < nw ? a.words[tile_word(s, w, capw)] : 0;
            for (int ch = 0; ch < nchunk; ++ch) {
                const int32_t lo = ch * pay, hi = min(total, lo + pay);
                __syncthreads();
                bwd_stage<T>(a, ta, tg, R, lo, hi, S);
                __syncthreads();
                // entries ascend within a word: entry 0 is its smallest slot,
                // entry 3 its largest
                while (w < nw && (int32_t)(cur & 0xFFFFu) < hi) {
                    const uint64_t nxt = w + LPA < nw ? a.words[tile_word(s, w + LPA, capw)] : 0;
                    bwd_word<T, true>(cur, lo, hi, xi, yi, zi, gxi, gyi, gzi, ti, S.xy, S.z,
                                      S.gxy, S.gz, S.t, c, ax, ay, az, sa, sb);
                    if ((int32_t)(cur >> 48) >= hi) break;  // continues in a later chunk
                    cur = nxt;
                    w += LPA;
                }
            }
        }
#pragma unroll
        for (int o = 1; o < LPA; o <<= 1) {
            ax += __shfl_xor(ax, o, kWave);
            ay += __shfl_xor(ay, o, kWave);
            az += __shfl_xor(az, o, kWave);
        }
        if (active && sub == 0) {
            a.gx[3 * u] = ax;
            a.gx[3 * u + 1] = ay;
            a.gx[3 * u + 2] = az;
        }
        // partner type 0's own sums
#pragma unroll
        for (int b = 1; b < T; ++b) {
            sa[0] -= sa[b];
            sb[0] -= sb[b];
        }
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
#pragma unroll
            for (int b = 0; b < T; ++b) {
                SA[tt * T + b] += ti == tt ? sa[b] : 0.0;
                SB[tt * T + b] += ti == tt ? sb[b] : 0.0;
            }
        }
    }
}

// LPA lanes per home atom, or with LPA = 0 the lanes chosen per tile from
// its home count (tiles of a batch differ widely in size).  One workgroup per
// tile (a persistent grid walking the tiles, as the force gather can use,
// measured 12% slower on a 512-system batch).  At least 4 waves per SIMD: two workgroups per compute unit, as the LDS stage allows
// (at most 128 VGPRs; left free, the compiler takes ~170 and only one
// workgroup fits, which measured 7-13% slower despite the few spills now).
template <int T, int LPA>
__global__ __launch_bounds__(kTileThreads, 4) void k_backward_tile(BwdTileArgs a, PairTab tab) {
    static_assert(LPA == 0 || LPA == 1 || LPA == 2 || LPA == 4 || LPA == 8, "lanes per atom");
    __shared__ TileLds L;
    __shared__ RowTab R;
    __shared__ BwdLds c;
    __shared__ BwdStage<T> S;
    static_assert(kTileThreads == 512, "the partial-sum reduction assumes 512 lanes");
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kTab; ++k) {
            c.rc2[k] = tab.rc2[k];
            c.lj1[k] = tab.lj1[k];
            c.lj2[k] = tab.lj2[k];
            c.ieps[k] = tab.eps[k] > 0.0 ? 1.0 / tab.eps[k] : 0.0;
            c.isig[k] = tab.sig[k] > 0.0 ? 1.0 / tab.sig[k] : 0.0;
        }
    }
    auto tile = [&](int64_t lb) {
        int64_t lbl = 0;
        const TileArgs ta = tile_args_of(a.t, lb, lbl);
        const TileGeom tg = tile_setup(ta, lbl, L, &R);
        const int32_t total = L.off[tg.ncells];
        const int32_t nh = tile_home_count(L, tg);
        // stencil chunks of `pay` slots, each staged with the null slot after it
        constexpr int32_t pay = kBwdChunk - 1;
        const int nchunk = total > pay ? (total + pay - 1) / pay : 1;
        if (nchunk == 1) {
            bwd_stage<T>(a, ta, tg, R, 0, total, S);
            __syncthreads();
        }
        double SA[T * T], SB[T * T];  // all home atoms of this lane: by type pair
#pragma unroll
        for (int b = 0; b < T * T; ++b) SA[b] = SB[b] = 0.0;
        if constexpr (LPA == 0) {
            const int lanes = tile_pass_lanes(nh);
            if (lanes == 8)
                bwd_rows<T, 8>(a, ta, tg, L, R, c, S, nh, total, nchunk, pay, SA, SB);
            else if (lanes == 4)
                bwd_rows<T, 4>(a, ta, tg, L, R, c, S, nh, total, nchunk, pay, SA, SB);
            else if (lanes == 2)
                bwd_rows<T, 2>(a, ta, tg, L, R, c, S, nh, total, nchunk, pay, SA, SB);
            else
                bwd_rows<T, 1>(a, ta, tg, L, R, c, S, nh, total, nchunk, pay, SA, SB);
        } else {
            bwd_rows<T, LPA>(a, ta, tg, L, R, c, S, nh, total, nchunk, pay, SA, SB);
        }
        // this lane's terms of the 2 T^2 parameter gradients:
        // d/d eps = (lj1 SA - lj2 SB) / (2 eps),
        // d/d sigma = (12 lj1 SA - 6 lj2 SB) / (2 sigma)
        constexpr int NV = 2 * T * T, NVP = (NV + 7) / 8 * 8;
        double val[NVP];
#pragma unroll
        for (int k = NV; k < NVP; ++k) val[k] = 0.0;
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
#pragma unroll
            for (int b = 0; b < T; ++b) {
                const int k = tt * T + b;
                const double l1 = c.lj1[k], l2 = c.lj2[k];
                val[2 * k] = 0.5 * c.ieps[k] * (l1 * SA[k] - l2 * SB[k]);
                val[2 * k + 1] = 0.5 * c.isig[k] * (12.0 * l1 * SA[k] - 6.0 * l2 * SB[k]);
            }
        }
        // per-block partials in a fixed order through LDS, eight values at a
        // time: sums of 8 lanes, then of 8 of those, then of the last 8 (the
        // stage is free once every wave is done with its rows)
        static_assert(sizeof(BwdStage<T>) >= sizeof(double) * (8 * kTileThreads + 8 * 64 + 64),
                      "reduction space");
        double *red = reinterpret_cast<double *>(&S);
        double *red2 = red + 8 * kTileThreads, *red3 = red2 + 8 * 64;
        const int tid = (int)threadIdx.x;
        __syncthreads();
#pragma unroll
        for (int v0 = 0; v0 < NV; v0 += 8) {
#pragma unroll
            for (int j = 0; j < 8; ++j) red[j * kTileThreads + tid] = val[v0 + j];
            __syncthreads();
            {
                const int j = tid >> 6, seg = tid & 63;
                double t = 0.0;
#pragma unroll
                for (int m = 0; m < 8; ++m) t += red[j * kTileThreads + seg * 8 + m];
                red2[j * 64 + seg] = t;
            }
            __syncthreads();
            if (tid < 64) {
                const int j = tid >> 3, seg = tid & 7;
                double t = 0.0;
#pragma unroll
                for (int m = 0; m < 8; ++m) t += red2[j * 64 + seg * 8 + m];
                red3[j * 8 + seg] = t;
            }
            __syncthreads();
            if (tid < 8 && v0 + tid < NV) {
                double t = 0.0;
#pragma unroll
                for (int m = 0; m < 8; ++m) t += red3[tid * 8 + m];
                a.partials[lb * kPartVals + v0 + tid] = t;
            }
            if (v0 + 8 < NV) __syncthreads();  // the next values reuse the space
        }
    };
    tile(xcd_remap(blockIdx.x, gridDim.x));
}

// One block per parameter value v: out = sum over blocks b of p[b][v], in a
// fixed order.
__global__ __launch_bounds__(kThreads) void k_param_reduce(const double *__restrict__ p,
                                                           int64_t nblocks, int ntypes,
                                                           double *__restrict__ geps,
                                                           double *__restrict__ gsig) {
    __shared__ double s[kThreads];
    const int v = (int)blockIdx.x;
    double t = 0.0;
    for (int64_t b = threadIdx.x; b < nblocks; b += kThreads) t += p[b * kPartVals + v];
    s[threadIdx.x] = t;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *dst = (v & 1) ? gsig : geps;
        if (dst) dst[v >> 1] = s[0];
    }
    (void)ntypes;
}

template <int T>
hipError_t launch_bwd_lpa(const BwdTileArgs &a, const PairTab &tab, int lpa, unsigned b,
                          hipStream_t s) {
    if (lpa == 8) k_backward_tile<T, 8><<<b, kTileThreads, 0, s>>>(a, tab);
    else if (lpa == 4) k_backward_tile<T, 4><<<b, kTileThreads, 0, s>>>(a, tab);
    else if (lpa == 2) k_backward_tile<T, 2><<<b, kTileThreads, 0, s>>>(a, tab);
    else if (lpa == 1) k_backward_tile<T, 1><<<b, kTileThreads, 0, s>>>(a, tab);
    else k_backward_tile<T, 0><<<b, kTileThreads, 0, s>>>(a, tab);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_backward(const double *x, const int32_t *type, int64_t n, const Box &box,
                           const PairTab &tab, const int32_t *numneigh, const uint32_t *neigh,
                           int cap, const double *gF, double *gx, double *partials,
                           int64_t *nblocks_out, hipStream_t s) {
    const int64_t blocks = (n + kThreads - 1) / kThreads;
    *nblocks_out = blocks;
    if (n <= 0) return hipSuccess;
    BwdArgs a{x, type, n, box, numneigh, neigh, cap, gF, gx, partials, nullptr, nullptr};
    const unsigned b = (unsigned)blocks;
    switch (tab.ntypes) {
        case 1: k_backward<1><<<b, kThreads, 0, s>>>(a, tab); break;
        case 2: k_backward<2><<<b, kThreads, 0, s>>>(a, tab); break;
        case 3: k_backward<3><<<b, kThreads, 0, s>>>(a, tab); break;
        default: k_backward<4><<<b, kThreads, 0, s>>>(a, tab); break;
    }
    return hipGetLastError();
}

hipError_t launch_backward_batch(const double *x, const int32_t *type, int64_t n,
                                 const BatchView &b, const PairTab &tab, const int32_t *numneigh,
                                 const uint32_t *neigh, int cap, const double *gF, double *gx,
                                 double *partials, int64_t *nblocks_out, hipStream_t s) {
    const int64_t blocks = (n + kThreads - 1) / kThreads;
    *nblocks_out = n > 0 ? blocks : 0;
    if (n <= 0) return hipSuccess;
    Box none{};
    BwdArgs a{x, type, n, none, numneigh, neigh, cap, gF, gx, partials, b.reps, b.rid};
    const unsigned nb = (unsigned)blocks;
    switch (tab.ntypes) {
        case 1: k_backward<1><<<nb, kThreads, 0, s>>>(a, tab); break;
        case 2: k_backward<2><<<nb, kThreads, 0, s>>>(a, tab); break;
        case 3: k_backward<3><<<nb, kThreads, 0, s>>>(a, tab); break;
        default: k_backward<4><<<nb, kThreads, 0, s>>>(a, tab); break;
    }
    return hipGetLastError();
}

hipError_t launch_backward_tiled(const TileArgs &t, const double *x, const int32_t *type,
                                 int64_t n, const PairTab &tab, const int32_t *numneigh,
                                 const void *neigh, int cap, int sorted, int lpa,
                                 const double *gF, double *gx, double *partials,
                                 int64_t *nblocks_out, hipStream_t s) {
    const int64_t blocks = tile_blocks(t);
    *nblocks_out = n > 0 ? blocks : 0;
    if (n <= 0) return hipSuccess;
    BwdTileArgs a{t, x, type, numneigh, static_cast<const uint64_t *>(neigh), tile_capw(cap),
                  sorted, gF, gx, partials};
    const unsigned b = (unsigned)blocks;
    switch (tab.ntypes) {
        case 1: return launch_bwd_lpa<1>(a, tab, lpa, b, s);
        case 2: return launch_bwd_lpa<2>(a, tab, lpa, b, s);
        case 3: return launch_bwd_lpa<3>(a, tab, lpa, b, s);
        default: return launch_bwd_lpa<4>(a, tab, lpa, b, s);
    }
}

hipError_t launch_param_grads(const double *partials, int64_t nblocks, int ntypes,
                              double *geps, double *gsig, hipStream_t s) {
    k_param_reduce<<<2 * ntypes * ntypes, kThreads, 0, s>>>(partials, nblocks, ntypes, geps, gsig);
    return hipGetLastError();
}

}  // namespace ljmd
