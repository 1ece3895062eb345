// C-ABI entry points of libljmd: argument checks (all before any HIP call),
// workspace and aux layouts, per-type-pair constants, the choice of list
// format, and the launch sequences of the neighbor build, the force and
// adjoint evaluations and the velocity-Verlet loop.  Declarations and the
// contract of every entry point: include/ljmd.h.
#include "ljmd.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "tile.hpp"

namespace {

using namespace ljmd;

thread_local std::string g_last_hip_error;

// ---- measurement hooks: HIP event pairs around each phase ----
struct Mark {
    int phase;
    hipEvent_t a, b;
};
struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<Mark> marks;
    hipEvent_t take() {
        if (pool.empty()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            return e;
        }
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
};
Profiler g_prof;

// Records a start event on construction and a stop event on stop() when
// profiling is on; a no-op otherwise.
class Phase {
  public:
    Phase(int phase, hipStream_t s) : phase_(phase), s_(s) {
        if (!g_prof.on) return;
        a_ = g_prof.take();
        if (a_ && hipEventRecord(a_, s_) != hipSuccess) a_ = nullptr;
    }
    void stop() {
        if (!g_prof.on || !a_ || done_) return;
        done_ = true;
        hipEvent_t b = g_prof.take();
        if (!b || hipEventRecord(b, s_) != hipSuccess) return;
        g_prof.marks.push_back(Mark{phase_, a_, b});
    }
    ~Phase() { stop(); }

  private:
    int phase_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr;
    bool done_ = false;
};

#define LJMD_TRY(expr)                                              \
    do {                                                            \
        const hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) {                                     \
            g_last_hip_error = hipGetErrorString(e_);               \
            return LJMD_EHIP;                                       \
        }                                                           \
    } while (0)

// LJMD_TRY inside a profiled phase on stream `s`.
#define LJMD_PHASED(phase, expr)        \
    do {                                \
        Phase ph_((phase), s);          \
        LJMD_TRY(expr);                 \
    } while (0)

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Checks the parameter tables; on success stores the largest neighbor cutoff.
int check_params(const ljmd_params *p, double *max_rnb) {
    if (!p) return LJMD_EINVAL;
    if (p->ntypes < 1) return LJMD_EINVAL;
    if (p->ntypes > LJMD_MAX_TYPES) return LJMD_ENOTSUP;
    if (!std::isfinite(p->skin) || p->skin < 0.0) return LJMD_EINVAL;
    double m = 0.0;
    for (int a = 0; a < p->ntypes; ++a) {
        for (int b = 0; b < p->ntypes; ++b) {
            if (!finite_pos(p->eps[a][b]) || !finite_pos(p->sigma[a][b]) ||
                !finite_pos(p->rc[a][b]))
                return LJMD_EINVAL;
            if (p->eps[a][b] != p->eps[b][a] || p->sigma[a][b] != p->sigma[b][a] ||
                p->rc[a][b] != p->rc[b][a])
                return LJMD_EINVAL;
            const double r = p->rc[a][b] + p->skin;
            if (r > m) m = r;
        }
    }
    *max_rnb = m;
    return LJMD_OK;
}

// Cell grid limits: int32 cell indices and cell-start tables of ncell + 1
// entries (the counts are compared in floating point, before any conversion).
constexpr double kMaxCellsPerDim = 1 << 20;
constexpr double kMaxCells = 2147483646.0;  // INT32_MAX - 1

int check_box(const ljmd_box *box, double max_rnb) {
    if (!box) return LJMD_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (!finite_pos(box->len[d]) || box->len[d] >= 1.0e9) return LJMD_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (box->len[d] < 2.0 * max_rnb) return LJMD_EBOX;
    double cells = 1.0;
    for (int d = 0; d < 3; ++d) {
        const double nc = std::floor(box->len[d] / (max_rnb * (1.0 + 1e-12)));
        if (!(nc <= kMaxCellsPerDim)) return LJMD_ENOTSUP;
        cells *= nc;
    }
    if (!(cells <= kMaxCells)) return LJMD_ENOTSUP;
    return LJMD_OK;
}

int check_n(int64_t n) {
    if (n < 0) return LJMD_EINVAL;
    if (n >= LJMD_MAX_ATOMS) return LJMD_ENOTSUP;
    return LJMD_OK;
}

Box make_box(const ljmd_box *b) {
    Box r;
    for (int d = 0; d < 3; ++d) {
        r.L[d] = b->len[d];
        r.hL[d] = 0.5 * b->len[d];
    }
    return r;
}

// Cells at least max_rnb * (1 + 1e-12) wide, so rounding in the binning can
// never put two atoms closer than the neighbor cutoff two cells apart.
Grid make_grid(const ljmd_box *b, double max_rnb) {
    Grid g;
    g.ncell = 1;
    for (int d = 0; d < 3; ++d) {
        int nc = (int)std::floor(b->len[d] / (max_rnb * (1.0 + 1e-12)));
        if (nc < 1) nc = 1;
        g.nc[d] = nc;
        g.cinv[d] = nc / b->len[d];
        g.ncell *= nc;
    }
    return g;
}

PairTab make_tab(const ljmd_params *p) {
    PairTab t;
    std::memset(&t, 0, sizeof(t));
    t.ntypes = p->ntypes;
    const int T = p->ntypes;
    for (int a = 0; a < T; ++a) {
        for (int b = 0; b < T; ++b) {
            const int k = a * T + b;
            const double e = p->eps[a][b], s = p->sigma[a][b], rc = p->rc[a][b];
            const double rn = rc + p->skin;
            const double s2 = s * s, s6 = s2 * s2 * s2, s12 = s6 * s6;
            t.rnb2[k] = rn * rn;
            t.rc2[k] = rc * rc;
            t.lj1[k] = 48.0 * e * s12;
            t.lj2[k] = 24.0 * e * s6;
            t.lj3[k] = 4.0 * e * s12;
            t.lj4[k] = 4.0 * e * s6;
            t.eps[k] = e;
            t.sig[k] = s;
            t.lj1f[k] = (float)t.lj1[k];
            t.lj2f[k] = (float)t.lj2[k];
            t.lj3f[k] = (float)t.lj3[k];
            t.lj4f[k] = (float)t.lj4[k];
        }
    }
    return t;
}

// Strip length of the global-format build (home cells per 256-thread
// workgroup along x): about 200 home atoms.
int global_strip(int64_t n, const Grid &g) {
    const double mean = g.ncell > 0 ? (double)n / (double)g.ncell : 0.0;
    const double want = mean > 0.0 ? 200.0 / mean : 30.0;  // clamped before the conversion
    int b = want >= 30.0 ? 30 : (want < 1.0 ? 1 : (int)want);
    if (b > g.nc[0]) b = g.nc[0];
    return b;
}

constexpr int kStageSlots = 2560;  // stencil slots the tiled kernels stage at once

// Lanes per home atom for a tile of about H home atoms: small tiles (chosen
// for small systems, so that there are enough workgroups to fill the GPU)
// share each row between 2, 4 or 8 lanes to fill the workgroup.
int tile_lanes(double H) {
    if (H <= kTileThreads / 8 * 1.125) return 8;
    if (H <= kTileThreads / 4 * 1.125) return 4;
    if (H <= kTileThreads / 2 * 1.125) return 2;
    return 1;
}

// Below this mean home count the tiled readers choose their lanes per tile
// (the relative spread of the home counts, 1/sqrt(H), is then large).
constexpr double kPerTileLanesBelow = 200.0;

// Lanes per home atom a reader chooses for a tile of exactly nh home atoms
// (the host mirror of tile_pass_lanes).
int pass_lanes(double nh) {
    if (nh <= kTileThreads / 8) return 8;
    if (nh <= kTileThreads / 4) return 4;
    if (nh <= kTileThreads / 2) return 2;
    return 1;
}

// Fraction of a workgroup's lanes kept busy by tiles of about H home atoms:
// with the lanes fixed for the whole list (1, 2 or 4, one pass covering H
// plus one standard deviation), or chosen per tile (averaged over home
// counts H - sd, H, H + sd).
double util_fixed(double H) {
    const int lanes = H <= kTileThreads / 4 * 1.125 ? 4 : (H <= kTileThreads / 2 * 1.125 ? 2 : 1);
    const double per = (double)(kTileThreads / lanes);
    const double passes = std::max(1.0, std::ceil((H + std::sqrt(H)) / per));
    return std::max(H, 1.0) / (passes * per);
}
double util_per_tile(double H) {
    const double sd = std::sqrt(H), w[3] = {0.25, 0.5, 0.25};
    double u = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double nh = std::max(1.0, std::round(H + (k - 1) * sd));
        u += w[k] * nh * pass_lanes(nh) / kTileThreads;
    }
    return u;
}

// Best tile under one cost model; returns the tile count (0 if none fits).
// The score is the lanes spent per home atom (1 / utilisation) plus a small
// charge for staging S / H atoms per home atom, scaled up when the tiles
// fill less than one round of 512 workgroups (two per compute unit), and,
// in the small-system model, by the waste of a partly filled second round:
// there a tile's time is mostly latency, so a last round costs a whole one.
int64_t tile_choose(double m, const Grid &g, bool small_model, int ext[3]) {
    double best = 1e300;
    int64_t best_blocks = 0;
    ext[0] = ext[1] = ext[2] = 1;
    for (int bz = 1; bz <= 4 && bz <= g.nc[2]; ++bz) {
        for (int by = 1; by <= 4 && by <= g.nc[1]; ++by) {
            const int rows = (by + 2) * (bz + 2);
            if (by * bz > kTileMaxHome || rows > kTileMaxRows) continue;
            for (int bx = 1; bx <= g.nc[0] && (bx + 2) * rows <= kTileMaxCells; ++bx) {
                const double H = bx * by * bz * m, S = (bx + 2) * rows * m;
                if (3.0 * S >= (double)kTileSlots) continue;
                const bool per_tile = small_model && H < kPerTileLanesBelow;
                const double util = per_tile ? util_per_tile(H) : util_fixed(H);
                const int64_t blocks = (int64_t)((g.nc[0] + bx - 1) / bx) *
                                       ((g.nc[1] + by - 1) / by) * ((g.nc[2] + bz - 1) / bz);
                double score = 1.0 / util + 0.01 * S / std::max(H, 1e-9);
                if (S + 3.0 * std::sqrt(S) > kStageSlots) score += 1.0;
                const double rounds = (double)blocks / 512.0;
                if (rounds < 1.0) score /= rounds;
                else if (small_model && rounds < 2.0) score *= 2.0 / rounds;
                if (score < best - 1e-9 || (score < best + 1e-9 && bx > ext[0])) {
                    best = score;
                    best_blocks = blocks;
                    ext[0] = bx;
                    ext[1] = by;
                    ext[2] = bz;
                }
            }
        }
    }
    return best_blocks;
}

// Tile extents of the tiled format (home cells per workgroup along x, y, z),
// from the mean cell occupancy m.  A workgroup has kTileThreads lanes; the
// home count H = cells * m should fill them at the chosen lanes per atom,
// the stencil (S atoms) should fit the kernels' staging buffer and leave the
// 16-bit slots three-fold headroom.  A system whose tiles would not fill one
// round of workgroups is re-tiled under the small-system model (lanes chosen
// per tile, partly filled rounds charged in full).  *ok is false when no
// tile meets the slot bound.
void tile_for(int64_t n, const Grid &g, int ext[3], bool *ok) {
    const double m = g.ncell > 0 ? (double)n / (double)g.ncell : 0.0;
    const int64_t blocks = tile_choose(m, g, false, ext);
    if (blocks > 0 && blocks < 512) tile_choose(m, g, true, ext);
    *ok = blocks > 0;
}

Workspace layout(int64_t n, const Grid &g, int64_t tblocks) {
    Workspace w;
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    const int64_t len = g.ncell + 1;
    const int64_t nscan = (len + kScanItems - 1) / kScanItems;
    w.scan_bsum = take(sizeof(int32_t) * (nscan + 1));
    w.atom_cell = take(sizeof(int32_t) * n);
    w.atom_slot = take(sizeof(int32_t) * n);
    w.tmp = take(sizeof(int32_t) * n);
    w.pos = take(sizeof(double) * 4 * n);
    const int64_t nb = (n + 255) / 256;
    w.part_a_blocks = (nb > tblocks ? nb : tblocks) + 1;
    w.part_a = take(sizeof(double) * kPartVals * w.part_a_blocks);
    w.part_b_blocks = (3 * n + 255) / 256 + 1;
    w.part_b = take(sizeof(double) * w.part_b_blocks);
    w.sort_v = take(sizeof(double) * 3 * n);
    w.sort_i = take(sizeof(int32_t) * 2 * n);
    w.xalt = take(sizeof(double) * 3 * n);
    w.total = off;
    return w;
}

Aux aux_layout(int64_t n, const Grid &g) {
    Aux a;
    a.perm = 0;
    a.cell_start = align256(sizeof(int32_t) * n);
    a.total = a.cell_start + align256(sizeof(int32_t) * (g.ncell + 1));
    return a;
}

struct Ctx {
    Box box;
    Grid g;
    PairTab tab;
    Workspace w;
    Aux aux;
    double max_rnb;
    int ext[3];     // tile extents of the tiled format
    bool slot_ok;   // a tile meets the 16-bit slot bound
    int strip;      // strip length of the global-format build
    int64_t tblocks;
};

int prepare(int64_t n, const ljmd_box *box, const ljmd_params *p, Ctx *c) {
    int rc = check_n(n);
    if (rc) return rc;
    rc = check_params(p, &c->max_rnb);
    if (rc) return rc;
    rc = check_box(box, c->max_rnb);
    if (rc) return rc;
    c->box = make_box(box);
    c->g = make_grid(box, c->max_rnb);
    c->tab = make_tab(p);
    tile_for(n, c->g, c->ext, &c->slot_ok);
    c->strip = global_strip(n, c->g);
    const int64_t tiles = (int64_t)((c->g.nc[0] + c->ext[0] - 1) / c->ext[0]) *
                          ((c->g.nc[1] + c->ext[1] - 1) / c->ext[1]) *
                          ((c->g.nc[2] + c->ext[2] - 1) / c->ext[2]);
    const int64_t strips = (int64_t)((c->g.nc[0] + c->strip - 1) / c->strip) * c->g.nc[1] *
                           c->g.nc[2];
    c->tblocks = std::max(tiles, strips);
    c->w = layout(n, c->g, c->tblocks);
    c->aux = aux_layout(n, c->g);
    return LJMD_OK;
}

int check_nlist(const ljmd_nlist *nl, int64_t n, const Ctx &c) {
    if (!nl) return LJMD_EINVAL;
    if (nl->n != n) return LJMD_EINVAL;
    if (nl->mode != LJMD_FULL && nl->mode != LJMD_HALF) return LJMD_EINVAL;
    if (nl->cap < 1) return LJMD_EINVAL;
    if (!nl->status) return LJMD_EINVAL;
    if (n > 0 && (!nl->numneigh || !nl->neigh || !nl->aux)) return LJMD_EINVAL;
    if (n > 0 && nl->aux_bytes < c.aux.total) return LJMD_EINVAL;
    return LJMD_OK;
}

// A list may be read only with the box and cutoffs it was built for.
int check_built(const ljmd_nlist *nl, const Ctx &c) {
    if (nl->format != LJMD_FMT_GLOBAL && nl->format != LJMD_FMT_TILED) return LJMD_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (nl->ncell[d] != c.g.nc[d]) return LJMD_EINVAL;
    const int *ext = nl->format == LJMD_FMT_TILED ? c.ext : nullptr;
    for (int d = 0; d < 3; ++d) {
        const int want = ext ? ext[d] : (d == 0 ? c.strip : 1);
        if (nl->tile[d] != want) return LJMD_EINVAL;
    }
    return LJMD_OK;
}

int check_ws(void *ws, size_t ws_bytes, const Workspace &w) {
    if (ws_bytes < w.total) return LJMD_EWORKSPACE;
    if (!ws) return LJMD_EINVAL;
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return LJMD_EINVAL;
    return LJMD_OK;
}

TileArgs tile_args(const Ctx &c, const ljmd_nlist *nl) {
    TileArgs t;
    std::memset(&t, 0, sizeof(t));  // single system: no batch table
    char *aux = static_cast<char *>(nl->aux);
    t.cell_start = reinterpret_cast<const int32_t *>(aux + c.aux.cell_start);
    t.perm = reinterpret_cast<const int32_t *>(aux + c.aux.perm);
    t.g = c.g;
    t.box = c.box;
    for (int d = 0; d < 3; ++d) {
        t.ext[d] = nl->tile[d];
        t.ntile[d] = (c.g.nc[d] + t.ext[d] - 1) / t.ext[d];
    }
    return t;
}

// Wrap and bin; with `sort`, also permute x, v, type and id into cell order
// (the binning's permutation then becomes the identity); then build the list
// in the tiled format when every dimension has 3 or more cells.
int build(double *x, const int32_t *type, int64_t n, const Ctx &c, ljmd_nlist *nl, char *ws,
          hipStream_t s, bool sort = false, double *v = nullptr, int32_t *type_mut = nullptr,
          int32_t *id = nullptr, double disp_lim2 = -1.0) {
    Phase ph(LJMD_PHASE_BUILD, s);
    const bool tiled = !(nl->flags & LJMD_NL_GLOBAL) && c.slot_ok && c.g.nc[0] >= 3 &&
                       c.g.nc[1] >= 3 && c.g.nc[2] >= 3;
    nl->format = tiled ? LJMD_FMT_TILED : LJMD_FMT_GLOBAL;
    nl->flags = sort ? (nl->flags | LJMD_NL_SORTED) : (nl->flags & ~LJMD_NL_SORTED);
    for (int d = 0; d < 3; ++d) {
        nl->ncell[d] = c.g.nc[d];
        nl->tile[d] = tiled ? c.ext[d] : (d == 0 ? c.strip : 1);
    }
    if (n <= 0) return LJMD_OK;
    char *aux = static_cast<char *>(nl->aux);
    int32_t *cell_start = reinterpret_cast<int32_t *>(aux + c.aux.cell_start);
    int32_t *perm = reinterpret_cast<int32_t *>(aux + c.aux.perm);
    LJMD_TRY(launch_bin(x, type, n, c.box, c.g, nl->xref, ws, c.w, cell_start, perm, s, nullptr,
                        nullptr, 0, disp_lim2, disp_lim2 >= 0.0 ? nl->status : nullptr, sort));
    if (sort) LJMD_TRY(launch_sort(n, x, v, type_mut, id, nl->xref, perm, ws, c.w, s));
    LJMD_TRY(launch_nl_build(n, tile_args(c, nl), c.tab, nl->mode == LJMD_HALF, tiled, ws, c.w,
                             nl->neigh, nl->numneigh, nl->cap, nl->status, s));
    return LJMD_OK;
}

// Lanes sharing one home atom's row in the tiled full-list gather and adjoint
// (ljmd_set_gather_lanes); 0: chosen from the list's tile size.
std::atomic<int> g_gather_lanes{0};

int list_lanes(const Ctx &c, const ljmd_nlist *nl) {
    const int set = g_gather_lanes.load();
    if (set) return set;
    const double m = c.g.ncell > 0 ? (double)nl->n / (double)c.g.ncell : 0.0;
    const double H = (double)nl->tile[0] * nl->tile[1] * nl->tile[2] * m;
    return H < kPerTileLanesBelow ? 0 : tile_lanes(H);  // 0: chosen per tile
}

// A list whose force kernel can apply the velocity-Verlet update itself: a
// full list in the tiled format (gather, each atom's force final in one lane).
bool fusable(const ljmd_nlist *nl) {
    return nl->format == LJMD_FMT_TILED && nl->mode == LJMD_FULL;
}

int forces(const double *x, const int32_t *type, int64_t n, const Ctx &c, const ljmd_nlist *nl,
           int mixed, int ev, double *f, char *ws, int64_t *nblocks, hipStream_t s,
           const Kick *kick = nullptr) {
    double *part = reinterpret_cast<double *>(ws + c.w.part_a);
    Phase ph(LJMD_PHASE_FORCE, s);
    if (nl->format == LJMD_FMT_TILED)
        LJMD_TRY(launch_forces_tiled(tile_args(c, nl), x, type, n, c.tab, nl->numneigh, nl->neigh,
                                     nl->cap, (nl->flags & LJMD_NL_SORTED) != 0,
                                     nl->mode == LJMD_HALF, mixed, ev, list_lanes(c, nl), f,
                                     part, nblocks, s, kick));
    else
        LJMD_TRY(launch_forces(x, type, n, c.box, c.tab, nl->numneigh, nl->neigh, nl->cap,
                               nl->mode == LJMD_HALF, mixed, ev, f, part, nblocks, s));
    return LJMD_OK;
}

// Argument checks of the adjoint (every one before any HIP call).
int check_backward(const double *x, const int32_t *type, int64_t n, const ljmd_box *box,
                   const ljmd_params *p, const ljmd_nlist *nl, const double *gF, uint32_t flags,
                   double *gx, Ctx *c) {
    int rc = prepare(n, box, p, c);
    if (rc) return rc;
    if ((rc = check_nlist(nl, n, *c))) return rc;
    if (nl->mode != LJMD_FULL) return LJMD_ENOTSUP;
    if (flags & LJMD_PREC_MIXED) return LJMD_ENOTSUP;
    if ((rc = check_built(nl, *c))) return rc;
    if (n > 0 && (!x || !gF || !gx)) return LJMD_EINVAL;
    if (n > 0 && p->ntypes > 1 && !type) return LJMD_EINVAL;
    return LJMD_OK;
}

// Workgroups of the adjoint launch, one row of kPartVals partials each: one
// per tile of a tiled list, one per 256 atoms of a global one.
int64_t backward_blocks(int64_t n, const Ctx &c, const ljmd_nlist *nl) {
    if (n <= 0) return 0;
    if (nl->format == LJMD_FMT_TILED) return tile_blocks(tile_args(c, nl));
    return (n + 255) / 256;
}

// The adjoint's launches, with its per-block partials in `part`.
int backward(const double *x, const int32_t *type, int64_t n, const ljmd_params *p,
             const ljmd_nlist *nl, const double *gF, double *gx, double *geps, double *gsig,
             const Ctx &c, double *part, hipStream_t s) {
    const int32_t *ty = p->ntypes > 1 ? type : nullptr;
    int64_t nb = 0;
    if (nl->format == LJMD_FMT_TILED)
        LJMD_PHASED(LJMD_PHASE_FORCE,
                    launch_backward_tiled(tile_args(c, nl), x, ty, n, c.tab, nl->numneigh,
                                          nl->neigh, nl->cap, (nl->flags & LJMD_NL_SORTED) != 0,
                                          g_gather_lanes.load(), gF, gx, part, &nb, s));
    else
        LJMD_PHASED(LJMD_PHASE_FORCE,
                    launch_backward(x, ty, n, c.box, c.tab, nl->numneigh, nl->neigh, nl->cap, gF,
                                    gx, part, &nb, s));
    if (geps || gsig)
        LJMD_PHASED(LJMD_PHASE_OTHER, launch_param_grads(part, nb, p->ntypes, geps, gsig, s));
    return LJMD_OK;
}

// ---- the allocation-free adjoint: its partials in a static device array ----
//
// `scratch` holds the adjoint's per-block partials for ljmd_lj_backward_noalloc
// (LJMD_NOALLOC_MAX_BLOCKS rows of kPartVals doubles, 4 MiB on every device
// the library runs on, held until the process ends).  In host code its name
// is only a stand-in for the device copy, so kernels get the device address
// that hipGetSymbolAddress returns, looked up once per device (with that
// device current) and kept.  Every block overwrites its own row before the
// reduction reads it, so nothing needs clearing between calls; calls that
// overlap on one device share the array and race.
constexpr int64_t kScratchBlocks = LJMD_NOALLOC_MAX_BLOCKS;
static __device__ __align__(256) double scratch[kScratchBlocks * kPartVals];

std::mutex g_scratch_mu;
std::vector<double *> g_scratch_ptr;  // device address of `scratch`, per device

int scratch_of_current_device(double **out) {
    int dev = 0;
    LJMD_TRY(hipGetDevice(&dev));
    if (dev < 0) return LJMD_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        LJMD_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return LJMD_EHIP;
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return LJMD_OK;
}

// ---- batches of independent systems ----

struct BatchCtx {
    int32_t nrep = 0;
    int64_t n = 0;           // atoms in the batch
    int64_t ncell = 0;       // cells of all systems
    int64_t nitems = 0;      // global-format build work items of all systems
    int64_t ntiles = 0;      // tiles of a tiled list of all systems (<= nitems)
    double max_rnb = 0.0;
    PairTab tab;
    Workspace w;             // the single-system layout sized for the batch
    size_t reps_off = 0;     // RepInfo[nrep]
    size_t rid_off = 0;      // int32[n]
    size_t ev_off = 0;       // double[7][n] per-atom energy / virial halves
    size_t bwd_off = 0;      // double[blocks][kPartVals] adjoint / force partials
    size_t tile_rep_off = 0; // int32[nitems + 1] (>= ntiles): system of each tile of a tiled list
    size_t total = 0;
    Aux aux;
    int tile_atoms = kBatchTileAtomsDefault;  // home atoms per tile (and build strip)
    double nbar = 0.0;       // expected neighbors per atom: (4 pi / 3) max_rnb^3 n / volume
};

// Host mirror of the device plan: grid, strip and tile rows of every system
// (the same functions as the plan kernel), for the totals.
int prepare_batch(const ljmd_batch *b, const ljmd_params *p, BatchCtx *c) {
    if (!b || b->nrep < 1 || !b->offsets || !b->boxes) return LJMD_EINVAL;
    int rc = check_params(p, &c->max_rnb);
    if (rc) return rc;
    if (b->offsets[0] != 0) return LJMD_EINVAL;
    if (b->tile_atoms != 0 && (b->tile_atoms < kBatchTileAtomsMin ||
                               b->tile_atoms > kBatchTileAtomsMax))
        return LJMD_EINVAL;
    c->tile_atoms = b->tile_atoms ? b->tile_atoms : kBatchTileAtomsDefault;
    c->nrep = b->nrep;
    double volume = 0.0;
    for (int32_t r = 0; r < b->nrep; ++r) {
        const int64_t na = b->offsets[r + 1] - b->offsets[r];
        if (na < 0) return LJMD_EINVAL;
        ljmd_box bx;
        for (int d = 0; d < 3; ++d) bx.len[d] = b->boxes[3 * r + d];
        if ((rc = check_box(&bx, c->max_rnb))) return rc;
        const Grid g = make_grid(&bx, c->max_rnb);
        volume += bx.len[0] * bx.len[1] * bx.len[2];
        const double mean = g.ncell > 0 ? (double)na / (double)g.ncell : 0.0;
        const int strip = batch_strip(mean, g.nc[0], c->tile_atoms);
        const int ey = batch_tile_rows(mean, strip, g.nc[1], c->tile_atoms);
        const int64_t nsx = (g.nc[0] + strip - 1) / strip;
        c->ncell += g.ncell;
        if ((double)c->ncell > kMaxCells) return LJMD_ENOTSUP;
        c->nitems += nsx * g.nc[1] * g.nc[2];
        c->ntiles += nsx * ((g.nc[1] + ey - 1) / ey) * g.nc[2];
    }
    c->n = b->offsets[b->nrep];
    if ((rc = check_n(c->n))) return rc;
    c->nbar = 4.18879020478639 * c->max_rnb * c->max_rnb * c->max_rnb * (double)c->n / volume;
    c->tab = make_tab(p);
    Grid all;
    all.nc[0] = all.nc[1] = all.nc[2] = 1;
    all.cinv[0] = all.cinv[1] = all.cinv[2] = 0.0;
    all.ncell = c->ncell;
    c->w = layout(c->n, all, c->nitems);
    size_t off = c->w.total;
    c->reps_off = off;
    off = align256(off + sizeof(RepInfo) * (size_t)c->nrep);
    c->rid_off = off;
    off = align256(off + sizeof(int32_t) * (size_t)c->n);
    c->ev_off = off;
    off = align256(off + sizeof(double) * 7 * (size_t)c->n);
    c->bwd_off = off;
    const int64_t pblocks = std::max<int64_t>((c->n + 255) / 256, c->nitems) + 1;
    off = align256(off + sizeof(double) * kPartVals * (size_t)pblocks);
    c->tile_rep_off = off;
    off = align256(off + sizeof(int32_t) * (size_t)(c->nitems + 1));
    c->total = off;
    c->aux = aux_layout(c->n, all);
    return LJMD_OK;
}

int check_batch_ws(void *ws, size_t ws_bytes, const BatchCtx &c) {
    if (ws_bytes < c.total) return LJMD_EWORKSPACE;
    if (!ws) return LJMD_EINVAL;
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return LJMD_EINVAL;
    return LJMD_OK;
}

int check_batch_nlist(const ljmd_nlist *nl, const BatchCtx &c) {
    if (!nl || nl->n != c.n || nl->mode != LJMD_FULL || nl->cap < 1 || !nl->status)
        return !nl || nl->mode == LJMD_FULL ? LJMD_EINVAL : LJMD_ENOTSUP;
    if (c.n > 0 && (!nl->numneigh || !nl->neigh || !nl->aux)) return LJMD_EINVAL;
    if (c.n > 0 && nl->aux_bytes < c.aux.total) return LJMD_EINVAL;
    return LJMD_OK;
}

// A batch list may be read only with the batch it was built for.
int check_batch_built(const ljmd_nlist *nl, const BatchCtx &c) {
    if (nl->format != LJMD_FMT_GLOBAL && nl->format != LJMD_FMT_TILED) return LJMD_EINVAL;
    if (!(nl->flags & LJMD_NL_BATCH)) return LJMD_EINVAL;
    if (nl->ncell[0] != (int32_t)c.ncell || nl->ncell[1] != c.nrep) return LJMD_EINVAL;
    if (nl->tile[0] != c.tile_atoms) return LJMD_EINVAL;  // built for another tiling
    return LJMD_OK;
}

// Device plan (per-system table and the system of every atom), written into
// the workspace at the start of every batch call.
BatchView batch_view(const ljmd_batch *b, const BatchCtx &c, char *ws) {
    BatchView v;
    v.nrep = c.nrep;
    v.offsets = b->d_offsets;
    v.reps = reinterpret_cast<const RepInfo *>(ws + c.reps_off);
    v.rid = reinterpret_cast<const int32_t *>(ws + c.rid_off);
    return v;
}

int batch_plan(const ljmd_batch *b, const BatchCtx &c, char *ws, hipStream_t s) {
    LJMD_PHASED(LJMD_PHASE_OTHER,
                launch_batch_plan(c.nrep, b->d_offsets, b->d_boxes, c.max_rnb, c.tile_atoms,
                                  reinterpret_cast<RepInfo *>(ws + c.reps_off),
                                  reinterpret_cast<int32_t *>(ws + c.rid_off), c.n,
                                  reinterpret_cast<int32_t *>(ws + c.tile_rep_off), c.ntiles,
                                  s));
    return LJMD_OK;
}

// Tile arguments of a tiled batch list: every system's tiles (a strip along
// x, ey cells along y), numbered through the plan's tile bases.
TileArgs batch_tile_args(const BatchCtx &c, const ljmd_nlist *nl, const char *ws) {
    TileArgs t;
    std::memset(&t, 0, sizeof(t));
    const char *aux = static_cast<const char *>(nl->aux);
    t.cell_start = reinterpret_cast<const int32_t *>(aux + c.aux.cell_start);
    t.perm = reinterpret_cast<const int32_t *>(aux + c.aux.perm);
    t.reps = reinterpret_cast<const RepInfo *>(ws + c.reps_off);
    t.tile_rep = reinterpret_cast<const int32_t *>(ws + c.tile_rep_off);
    t.nbatch = c.ntiles;
    return t;
}

int batch_build(double *x, const int32_t *type, const ljmd_batch *b, const BatchCtx &c,
                ljmd_nlist *nl, char *ws, hipStream_t s, bool sort = false, double *v = nullptr,
                int32_t *type_mut = nullptr, int32_t *id = nullptr, double disp_lim2 = -1.0) {
    Phase ph(LJMD_PHASE_BUILD, s);
    const bool tiled = !(nl->flags & LJMD_NL_GLOBAL);
    nl->format = tiled ? LJMD_FMT_TILED : LJMD_FMT_GLOBAL;
    nl->flags = (nl->flags | LJMD_NL_BATCH) & ~LJMD_NL_SORTED;
    if (sort) nl->flags |= LJMD_NL_SORTED;
    nl->ncell[0] = (int32_t)c.ncell;
    nl->ncell[1] = c.nrep;
    nl->ncell[2] = 0;
    nl->tile[0] = c.tile_atoms;
    nl->tile[1] = nl->tile[2] = 0;
    if (c.n <= 0) return LJMD_OK;
    const BatchView bv = batch_view(b, c, ws);
    char *aux = static_cast<char *>(nl->aux);
    int32_t *cell_start = reinterpret_cast<int32_t *>(aux + c.aux.cell_start);
    int32_t *perm = reinterpret_cast<int32_t *>(aux + c.aux.perm);
    Box none{};
    Grid gnone{};
    LJMD_TRY(launch_bin(x, type, c.n, none, gnone, nl->xref, ws, c.w, cell_start, perm, s, bv.reps,
                        bv.rid, c.ncell, disp_lim2, disp_lim2 >= 0.0 ? nl->status : nullptr,
                        sort));
    if (sort) LJMD_TRY(launch_sort(c.n, x, v, type_mut, id, nl->xref, perm, ws, c.w, s));
    if (tiled)
        LJMD_TRY(launch_nl_build(c.n, batch_tile_args(c, nl, ws), c.tab, 0, 1, ws, c.w, nl->neigh,
                                 nl->numneigh, nl->cap, nl->status, s));
    else
        LJMD_TRY(launch_nl_build_batch(c.n, bv, c.nitems, cell_start, perm, c.tab, 0, ws, c.w,
                                       nl->neigh, nl->numneigh, nl->cap, nl->status, s));
    return LJMD_OK;
}

// Force-kernel variant per batch class, set by the autotuner or the caller:
// keyed by the atom count (power-of-two bucket), the expected neighbors per
// atom (bucket of 8), the tile target of the list, the precision and the
// list format, so that batches of one workload class share a tuning.  The
// default is lanes chosen per tile on a tiled list, one lane per atom on a
// global one, 256-lane workgroups, one workgroup per tile or group of atoms.
struct TuneKey {
    int n_bucket;
    int nbar_bucket;
    int tile_atoms;
    int32_t mixed;
    int32_t format;
    bool operator<(const TuneKey &o) const {
        if (n_bucket != o.n_bucket) return n_bucket < o.n_bucket;
        if (nbar_bucket != o.nbar_bucket) return nbar_bucket < o.nbar_bucket;
        if (tile_atoms != o.tile_atoms) return tile_atoms < o.tile_atoms;
        return mixed != o.mixed ? mixed < o.mixed : format < o.format;
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, ljmd_batch_tuning> g_tune;

TuneKey tune_key(const BatchCtx &c, int mixed, int format) {
    int nb = 0;
    while (nb < 62 && (int64_t(1) << (nb + 1)) <= c.n) ++nb;
    const double q = c.nbar / 8.0;
    return TuneKey{nb, q < 1e6 ? (int)q : 1000000, c.tile_atoms, mixed, format};
}

ljmd_batch_tuning tuning_for(const BatchCtx &c, int mixed, int format) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(c, mixed, format));
    if (it != g_tune.end()) return it->second;
    if (format == LJMD_FMT_TILED) return ljmd_batch_tuning{0, 256, 0, c.tile_atoms};
    return ljmd_batch_tuning{1, 256, 0, c.tile_atoms};
}

bool tuning_valid(const ljmd_batch_tuning &t) {
    return (t.lanes_per_atom == 0 || t.lanes_per_atom == 1 || t.lanes_per_atom == 2 ||
            t.lanes_per_atom == 4) &&
           (t.block == 128 || t.block == 256) && t.persistent >= 0 && t.persistent <= 64;
}

int batch_forces(const double *x, const int32_t *type, const ljmd_batch *b, const BatchCtx &c,
                 const ljmd_nlist *nl, int mixed, bool ev, double *f, char *ws, hipStream_t s,
                 const ljmd_batch_tuning *force_cfg = nullptr, const Kick *kick = nullptr,
                 const FmOut *fm = nullptr) {
    const BatchView bv = batch_view(b, c, ws);
    const ljmd_batch_tuning t = force_cfg ? *force_cfg : tuning_for(c, mixed, nl->format);
    double *eva = ev ? reinterpret_cast<double *>(ws + c.ev_off) : nullptr;
    if (nl->format == LJMD_FMT_TILED) {
        // one workgroup per tile of every system, or a persistent grid walking
        // the tiles; the lanes per atom and the persistence of the tuning apply
        int64_t nb = 0;
        LJMD_PHASED(LJMD_PHASE_FORCE,
                    launch_forces_tiled(batch_tile_args(c, nl, ws), x, type, c.n, c.tab,
                                        nl->numneigh, nl->neigh, nl->cap,
                                        (nl->flags & LJMD_NL_SORTED) != 0, 0, mixed, ev,
                                        t.lanes_per_atom, f,
                                        reinterpret_cast<double *>(ws + c.bwd_off), &nb, s,
                                        kick, eva, t.persistent, fm));
        return LJMD_OK;
    }
    // the global-format kernel cannot apply the force-matching gradient
    // itself: forces first (into f, else a workspace buffer), then g
    double *fo = f;
    if (fm && !fo) fo = reinterpret_cast<double *>(ws + c.w.sort_v);
    LJMD_PHASED(LJMD_PHASE_FORCE,
                launch_forces_batch(x, type, c.n, bv, c.tab, nl->numneigh, nl->neigh, nl->cap,
                                    mixed, fo, eva, t.lanes_per_atom ? t.lanes_per_atom : 1,
                                    t.block, t.persistent, s));
    if (fm) LJMD_PHASED(LJMD_PHASE_OTHER, launch_fm_grad(fo, *fm, c.n, bv.reps, bv.rid, s));
    return LJMD_OK;
}

}  // namespace

extern "C" {

int64_t ljmd_nlist_entries(int64_t n, int32_t cap) {
    if (n < 0 || cap < 1) return 0;
    return ((n + 63) / 64) * 64 * (((int64_t)cap + 15) / 16 * 16);
}

size_t ljmd_workspace_bytes(int64_t n, const ljmd_box *box, const ljmd_params *p,
                            uint32_t flags) {
    (void)flags;
    Ctx c;
    if (prepare(n, box, p, &c) != LJMD_OK) return 0;
    return c.w.total;
}

size_t ljmd_nlist_aux_bytes(int64_t n, const ljmd_box *box, const ljmd_params *p) {
    Ctx c;
    if (prepare(n, box, p, &c) != LJMD_OK) return 0;
    return c.aux.total;
}

int ljmd_nl_build(double *x, const int32_t *type, int64_t n, const ljmd_box *box,
                  const ljmd_params *p, ljmd_nlist *nl, void *ws, size_t ws_bytes,
                  void *stream) {
    Ctx c;
    int rc = prepare(n, box, p, &c);
    if (rc) return rc;
    if ((rc = check_nlist(nl, n, c))) return rc;
    if (n > 0 && !x) return LJMD_EINVAL;
    if (n > 0 && p->ntypes > 1 && !type) return LJMD_EINVAL;
    if ((rc = check_ws(ws, ws_bytes, c.w))) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    LJMD_PHASED(LJMD_PHASE_OTHER, launch_set_i32(nl->status, LJMD_STATUS_WORDS, 0, s));
    return build(x, p->ntypes > 1 ? type : nullptr, n, c, nl, static_cast<char *>(ws), s);
}

namespace {
int export_list(const ljmd_nlist *nl, uint32_t *out, int32_t *counts, void *stream, int kmajor) {
    if (!nl || nl->n < 0 || nl->cap < 1) return LJMD_EINVAL;
    if (nl->n > 0 && (!out || !counts || !nl->numneigh || !nl->neigh)) return LJMD_EINVAL;
    if (nl->format != LJMD_FMT_GLOBAL && nl->format != LJMD_FMT_TILED) return LJMD_EINVAL;
    // a tiled batch list needs its batch (ljmd_batch_nl_export)
    if (nl->format == LJMD_FMT_TILED && (nl->flags & LJMD_NL_BATCH)) return LJMD_EINVAL;
    if (nl->n == 0) return LJMD_OK;
    TileArgs t;
    std::memset(&t, 0, sizeof(t));
    if (nl->format == LJMD_FMT_TILED) {
        if (!nl->aux) return LJMD_EINVAL;
        Grid g;
        g.ncell = 1;
        for (int d = 0; d < 3; ++d) {
            if (nl->ncell[d] < 3) return LJMD_EINVAL;
            g.nc[d] = nl->ncell[d];
            g.cinv[d] = 0.0;
            g.ncell *= nl->ncell[d];
        }
        const Aux a = aux_layout(nl->n, g);
        if (nl->aux_bytes < a.total) return LJMD_EINVAL;
        const char *aux = static_cast<const char *>(nl->aux);
        t.cell_start = reinterpret_cast<const int32_t *>(aux + a.cell_start);
        t.perm = reinterpret_cast<const int32_t *>(aux + a.perm);
        t.g = g;
        int rows = 1, home = 1;
        for (int d = 0; d < 3; ++d) {
            if (nl->tile[d] < 1 || nl->tile[d] > nl->ncell[d]) return LJMD_EINVAL;
            t.ext[d] = nl->tile[d];
            t.ntile[d] = (g.nc[d] + t.ext[d] - 1) / t.ext[d];
            if (d > 0) {
                rows *= t.ext[d] + 2;
                home *= t.ext[d];
            }
        }
        if (rows > kTileMaxRows || home > kTileMaxHome || (t.ext[0] + 2) * rows > kTileMaxCells)
            return LJMD_EINVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    LJMD_PHASED(LJMD_PHASE_OTHER,
                launch_nl_export(nl->n, t, nl->format == LJMD_FMT_TILED, nl->neigh, nl->numneigh,
                                 nl->cap, out, counts, s, kmajor));
    return LJMD_OK;
}
}  // namespace

int ljmd_nl_export(const ljmd_nlist *nl, uint32_t *out, int32_t *counts, void *stream) {
    return export_list(nl, out, counts, stream, 0);
}

int ljmd_nl_export_indices(const ljmd_nlist *nl, int32_t *out, int32_t *counts, void *stream) {
    return export_list(nl, reinterpret_cast<uint32_t *>(out), counts, stream, 1);
}

int ljmd_lj_forces(const double *x, const int32_t *type, int64_t n, const ljmd_box *box,
                   const ljmd_params *p, const ljmd_nlist *nl, uint32_t flags, double *f,
                   double *ev, void *ws, size_t ws_bytes, void *stream) {
    Ctx c;
    int rc = prepare(n, box, p, &c);
    if (rc) return rc;
    if ((rc = check_nlist(nl, n, c))) return rc;
    if ((rc = check_built(nl, c))) return rc;
    if (n > 0 && (!x || !f)) return LJMD_EINVAL;
    if (n > 0 && p->ntypes > 1 && !type) return LJMD_EINVAL;
    if ((rc = check_ws(ws, ws_bytes, c.w))) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    const int want_ev = (flags & LJMD_EV) && ev;
    int64_t nb = 0;
    if ((rc = forces(x, p->ntypes > 1 ? type : nullptr, n, c, nl, (flags & LJMD_PREC_MIXED) != 0,
                     want_ev, f, w, &nb, s)))
        return rc;
    if (want_ev)
        LJMD_PHASED(LJMD_PHASE_OTHER,
                    launch_reduce_partials(reinterpret_cast<double *>(w + c.w.part_a), nb, 7, ev,
                                           s));
    return LJMD_OK;
}

int ljmd_lj_backward(const double *x, const int32_t *type, int64_t n, const ljmd_box *box,
                     const ljmd_params *p, const ljmd_nlist *nl, const double *gF,
                     uint32_t flags, double *gx, double *geps, double *gsig, void *ws,
                     size_t ws_bytes, void *stream) {
    Ctx c;
    int rc = check_backward(x, type, n, box, p, nl, gF, flags, gx, &c);
    if (rc) return rc;
    if ((rc = check_ws(ws, ws_bytes, c.w))) return rc;
    double *part = reinterpret_cast<double *>(static_cast<char *>(ws) + c.w.part_a);
    return backward(x, type, n, p, nl, gF, gx, geps, gsig, c, part,
                    reinterpret_cast<hipStream_t>(stream));
}

int ljmd_lj_backward_noalloc(const double *x, const int32_t *type, int64_t n,
                             const ljmd_box *box, const ljmd_params *p, const ljmd_nlist *nl,
                             const double *gF, uint32_t flags, double *gx, double *geps,
                             double *gsig, void *stream) {
    Ctx c;
    int rc = check_backward(x, type, n, box, p, nl, gF, flags, gx, &c);
    if (rc) return rc;
    if (backward_blocks(n, c, nl) > kScratchBlocks) return LJMD_ESCRATCH;
    double *part = nullptr;
    if ((rc = scratch_of_current_device(&part))) return rc;
    return backward(x, type, n, p, nl, gF, gx, geps, gsig, c, part,
                    reinterpret_cast<hipStream_t>(stream));
}

int ljmd_fm_grad(const double *x, const int32_t *type, int64_t n, const ljmd_box *box,
                 const ljmd_params *p, const ljmd_nlist *nl, const double *f_target,
                 const double *weight, uint32_t flags, double *f, double *gx, double *geps,
                 double *gsig, void *ws, size_t ws_bytes, void *stream) {
    Ctx c;
    // the forward may run in mixed precision; the adjoint is FP64
    int rc = check_backward(x, type, n, box, p, nl, f_target, flags & ~LJMD_PREC_MIXED, gx, &c);
    if (rc) return rc;
    if ((rc = check_ws(ws, ws_bytes, c.w))) return rc;
    if (n <= 0) return LJMD_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    double *g = reinterpret_cast<double *>(w + c.w.xalt);
    double *part = reinterpret_cast<double *>(w + c.w.part_a);
    const int32_t *ty = p->ntypes > 1 ? type : nullptr;
    const int mixed = (flags & LJMD_PREC_MIXED) != 0;
    const FmOut fm{f_target, weight, g};
    int64_t nb = 0;
    if (nl->format == LJMD_FMT_TILED) {
        LJMD_PHASED(LJMD_PHASE_FORCE,
                    launch_forces_tiled(tile_args(c, nl), x, ty, n, c.tab, nl->numneigh,
                                        nl->neigh, nl->cap, (nl->flags & LJMD_NL_SORTED) != 0, 0,
                                        mixed, 0, list_lanes(c, nl), f, part, &nb, s, nullptr,
                                        nullptr, 0, &fm));
    } else {
        double *fo = f ? f : reinterpret_cast<double *>(w + c.w.sort_v);
        LJMD_PHASED(LJMD_PHASE_FORCE,
                    launch_forces(x, ty, n, c.box, c.tab, nl->numneigh, nl->neigh, nl->cap, 0,
                                  mixed, 0, fo, part, &nb, s));
        LJMD_PHASED(LJMD_PHASE_OTHER, launch_fm_grad(fo, fm, n, nullptr, nullptr, s));
    }
    return backward(x, type, n, p, nl, g, gx, geps, gsig, c, part, s);
}

int ljmd_md_step(double *x, double *v, double *f, int32_t *type, int32_t *id, int64_t n,
                 const ljmd_box *box, const ljmd_params *p, ljmd_nlist *nl, double dt,
                 int64_t step0, int64_t nsteps, int32_t rebuild_every, int32_t thermo_every,
                 uint32_t flags, double *thermo, void *ws, size_t ws_bytes, void *stream) {
    Ctx c;
    int rc = prepare(n, box, p, &c);
    if (rc) return rc;
    if ((rc = check_nlist(nl, n, c))) return rc;
    if (!std::isfinite(dt) || dt <= 0.0) return LJMD_EINVAL;
    if (nsteps < 0 || rebuild_every < 1 || thermo_every < 0 || step0 < 0) return LJMD_EINVAL;
    if (n > 0 && (!x || !v || !f)) return LJMD_EINVAL;
    if (n > 0 && p->ntypes > 1 && !type) return LJMD_EINVAL;
    if (thermo_every > 0 && !thermo) return LJMD_EINVAL;
    if (!(flags & LJMD_SETUP) && (rc = check_built(nl, c))) return rc;
    double dtf[LJMD_MAX_TYPES] = {0, 0, 0, 0};
    for (int t = 0; t < p->ntypes; ++t) {
        if (!finite_pos(p->mass[t])) return LJMD_EINVAL;
        dtf[t] = 0.5 * dt / p->mass[t];
    }
    if ((rc = check_ws(ws, ws_bytes, c.w))) return rc;

    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    int32_t *ty = p->ntypes > 1 ? type : nullptr;
    const bool sort = (flags & LJMD_SORT) != 0;
    const int mixed = (flags & LJMD_PREC_MIXED) != 0;
    double *evp = reinterpret_cast<double *>(w + c.w.part_a);
    double *kep = reinterpret_cast<double *>(w + c.w.part_b);
    const double half_skin = 0.5 * p->skin;
    int64_t row = 0, nbf = 0, nbk = 0;

    auto overflowed = [&](bool *out) -> int {
        int32_t st_host[LJMD_STATUS_WORDS];
        LJMD_TRY(hipMemcpyAsync(st_host, nl->status, sizeof(st_host), hipMemcpyDeviceToHost, s));
        LJMD_TRY(hipStreamSynchronize(s));
        *out = st_host[LJMD_ST_OVERFLOW] != 0;
        return LJMD_OK;
    };
    bool ovf = false;
    LJMD_PHASED(LJMD_PHASE_OTHER, launch_set_i32(nl->status, LJMD_STATUS_WORDS, 0, s));
    if (flags & LJMD_SETUP) {
        const int th = thermo_every > 0 && step0 % thermo_every == 0;
        if ((rc = build(x, ty, n, c, nl, w, s, sort, v, ty, id))) return rc;
        if (flags & LJMD_SYNC_CHECK) {
            if ((rc = overflowed(&ovf))) return rc;
            if (ovf) return LJMD_ENEIGH_OVERFLOW;
        }
        if ((rc = forces(x, ty, n, c, nl, mixed, th, f, w, &nbf, s))) return rc;
        if (th) {
            // kinetic energy of the current velocities: a kick with zero
            // step leaves v unchanged and sums m v^2 / 2
            const double zero[LJMD_MAX_TYPES] = {0, 0, 0, 0};
            LJMD_PHASED(LJMD_PHASE_INTEGRATE,
                        launch_kick(x, v, f, ty, n, zero, p->mass, p->ntypes, dt, 0, 1, kep,
                                    &nbk, nl->status, s));
            LJMD_PHASED(LJMD_PHASE_OTHER,
                        launch_thermo_row(evp, nbf, kep, nbk, step0, thermo + 9 * row, s));
            ++row;
        }
    }
    if (nsteps == 0) return LJMD_OK;
    // With a full tiled list the gather applies the second half kick of a
    // step, and the next step's half kick and drift, as each atom's force is
    // done; the drifted positions go to the other of two buffers (the user's
    // x and a workspace copy), and the last positions are copied back to x
    // if they ended in the workspace copy.  The buffers change at every step
    // but the last, so when that is an odd number of times the first drift
    // already goes to the workspace copy and the last positions land in x.
    double *xc = x;
    double *xo = reinterpret_cast<double *>(w + c.w.xalt);
    if (fusable(nl) && !(flags & LJMD_SEPARATE_KICK) && (nsteps - 1) % 2 == 1) std::swap(xc, xo);
    LJMD_PHASED(LJMD_PHASE_INTEGRATE,
                launch_kick_drift(x, v, f, ty, n, dtf, p->ntypes, dt, s, xc));
    for (int64_t st = 1; st <= nsteps; ++st) {
        const int64_t g = step0 + st;
        if (g % rebuild_every == 0) {
            // the binning first checks the displacements since the last build
            if ((rc = build(xc, ty, n, c, nl, w, s, sort, v, ty, id, half_skin * half_skin)))
                return rc;
            if (flags & LJMD_SYNC_CHECK) {
                if ((rc = overflowed(&ovf))) {
                    if (xc != x) (void)hipMemcpyAsync(x, xc, sizeof(double) * 3 * n,
                                                      hipMemcpyDeviceToDevice, s);
                    return rc;
                }
                if (ovf) {
                    if (xc != x)
                        LJMD_TRY(hipMemcpyAsync(x, xc, sizeof(double) * 3 * n,
                                                hipMemcpyDeviceToDevice, s));
                    return LJMD_ENEIGH_OVERFLOW;
                }
            }
        }
        const int th = thermo_every > 0 && g % thermo_every == 0;
        if (fusable(nl) && !(flags & LJMD_SEPARATE_KICK)) {
            Kick k;
            k.v = v;
            k.xnext = xo;
            k.status = nl->status;
            for (int t = 0; t < kMaxTypes; ++t) {
                k.h[t] = t < p->ntypes ? dtf[t] : 0.0;
                k.mass[t] = t < p->ntypes ? p->mass[t] : 0.0;
            }
            k.dt = dt;
            k.mode = st < nsteps ? 2 : 1;
            if ((rc = forces(xc, ty, n, c, nl, mixed, th, f, w, &nbf, s, &k))) return rc;
            if (th) {
                LJMD_PHASED(LJMD_PHASE_OTHER,
                            launch_thermo_row(evp, nbf, nullptr, 0, g, thermo + 9 * row, s));
                ++row;
            }
            if (k.mode == 2) std::swap(xc, xo);
        } else {
            if ((rc = forces(xc, ty, n, c, nl, mixed, th, f, w, &nbf, s))) return rc;
            LJMD_PHASED(LJMD_PHASE_INTEGRATE,
                        launch_kick(xc, v, f, ty, n, dtf, p->mass, p->ntypes, dt, st < nsteps, th,
                                    kep, &nbk, nl->status, s));
            if (th) {
                LJMD_PHASED(LJMD_PHASE_OTHER,
                            launch_thermo_row(evp, nbf, kep, nbk, g, thermo + 9 * row, s));
                ++row;
            }
        }
    }
    if (xc != x)
        LJMD_PHASED(LJMD_PHASE_INTEGRATE,
                    hipMemcpyAsync(x, xc, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, s));
    return LJMD_OK;
}

// ---- batches ----

size_t ljmd_batch_workspace_bytes(const ljmd_batch *b, const ljmd_params *p, uint32_t flags) {
    (void)flags;
    BatchCtx c;
    if (prepare_batch(b, p, &c) != LJMD_OK) return 0;
    return c.total;
}

size_t ljmd_batch_aux_bytes(const ljmd_batch *b, const ljmd_params *p) {
    BatchCtx c;
    if (prepare_batch(b, p, &c) != LJMD_OK) return 0;
    return c.aux.total;
}

int ljmd_batch_nl_build(double *x, const int32_t *type, const ljmd_batch *b,
                        const ljmd_params *p, ljmd_nlist *nl, void *ws, size_t ws_bytes,
                        void *stream) {
    BatchCtx c;
    int rc = prepare_batch(b, p, &c);
    if (rc) return rc;
    if ((rc = check_batch_nlist(nl, c))) return rc;
    if (!b->d_offsets || !b->d_boxes) return LJMD_EINVAL;
    if (c.n > 0 && !x) return LJMD_EINVAL;
    if (c.n > 0 && p->ntypes > 1 && !type) return LJMD_EINVAL;
    if ((rc = check_batch_ws(ws, ws_bytes, c))) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    LJMD_PHASED(LJMD_PHASE_OTHER, launch_set_i32(nl->status, LJMD_STATUS_WORDS, 0, s));
    if ((rc = batch_plan(b, c, w, s))) return rc;
    return batch_build(x, p->ntypes > 1 ? type : nullptr, b, c, nl, w, s);
}

int ljmd_batch_nl_export(const ljmd_nlist *nl, const ljmd_batch *b, const ljmd_params *p,
                         uint32_t *out, int32_t *counts, void *ws, size_t ws_bytes,
                         void *stream) {
    BatchCtx c;
    int rc = prepare_batch(b, p, &c);
    if (rc) return rc;
    if ((rc = check_batch_nlist(nl, c))) return rc;
    if ((rc = check_batch_built(nl, c))) return rc;
    if (!b->d_offsets || !b->d_boxes) return LJMD_EINVAL;
    if (c.n > 0 && (!out || !counts)) return LJMD_EINVAL;
    if ((rc = check_batch_ws(ws, ws_bytes, c))) return rc;
    if (c.n == 0) return LJMD_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    if ((rc = batch_plan(b, c, w, s))) return rc;
    TileArgs t = batch_tile_args(c, nl, w);
    LJMD_PHASED(LJMD_PHASE_OTHER,
                launch_nl_export(c.n, t, nl->format == LJMD_FMT_TILED, nl->neigh, nl->numneigh,
                                 nl->cap, out, counts, s));
    return LJMD_OK;
}

int ljmd_batch_lj_forces(const double *x, const int32_t *type, const ljmd_batch *b,
                         const ljmd_params *p, const ljmd_nlist *nl, uint32_t flags, double *f,
                         double *ev, void *ws, size_t ws_bytes, void *stream) {
    BatchCtx c;
    int rc = prepare_batch(b, p, &c);
    if (rc) return rc;
    if ((rc = check_batch_nlist(nl, c))) return rc;
    if ((rc = check_batch_built(nl, c))) return rc;
    if (!b->d_offsets || !b->d_boxes) return LJMD_EINVAL;
    if (c.n > 0 && (!x || !f)) return LJMD_EINVAL;
    if (c.n > 0 && p->ntypes > 1 && !type) return LJMD_EINVAL;
    if ((rc = check_batch_ws(ws, ws_bytes, c))) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    const bool want_ev = (flags & LJMD_EV) && ev;
    if ((rc = batch_plan(b, c, w, s))) return rc;
    if ((rc = batch_forces(x, p->ntypes > 1 ? type : nullptr, b, c, nl,
                           (flags & LJMD_PREC_MIXED) != 0, want_ev, f, w, s)))
        return rc;
    if (want_ev)
        LJMD_PHASED(LJMD_PHASE_OTHER,
                    launch_batch_thermo(batch_view(b, c, w), nullptr, nullptr, nullptr,
                                        p->ntypes, reinterpret_cast<double *>(w + c.ev_off), c.n,
                                        0, nullptr, ev, s));
    return LJMD_OK;
}

int ljmd_batch_lj_backward(const double *x, const int32_t *type, const ljmd_batch *b,
                           const ljmd_params *p, const ljmd_nlist *nl, const double *gF,
                           uint32_t flags, double *gx, double *geps, double *gsig, void *ws,
                           size_t ws_bytes, void *stream) {
    BatchCtx c;
    int rc = prepare_batch(b, p, &c);
    if (rc) return rc;
    if ((rc = check_batch_nlist(nl, c))) return rc;
    if (flags & LJMD_PREC_MIXED) return LJMD_ENOTSUP;
    if ((rc = check_batch_built(nl, c))) return rc;
    if (!b->d_offsets || !b->d_boxes) return LJMD_EINVAL;
    if (c.n > 0 && (!x || !gF || !gx)) return LJMD_EINVAL;
    if (c.n > 0 && p->ntypes > 1 && !type) return LJMD_EINVAL;
    if ((rc = check_batch_ws(ws, ws_bytes, c))) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    double *part = reinterpret_cast<double *>(w + c.bwd_off);
    int64_t nb = 0;
    if ((rc = batch_plan(b, c, w, s))) return rc;
    if (nl->format == LJMD_FMT_TILED)
        LJMD_PHASED(LJMD_PHASE_FORCE,
                    launch_backward_tiled(batch_tile_args(c, nl, w), x,
                                          p->ntypes > 1 ? type : nullptr, c.n, c.tab,
                                          nl->numneigh, nl->neigh, nl->cap,
                                          (nl->flags & LJMD_NL_SORTED) != 0,
                                          g_gather_lanes.load(), gF, gx, part, &nb, s));
    else
        LJMD_PHASED(LJMD_PHASE_FORCE,
                    launch_backward_batch(x, p->ntypes > 1 ? type : nullptr, c.n,
                                          batch_view(b, c, w), c.tab, nl->numneigh, nl->neigh,
                                          nl->cap, gF, gx, part, &nb, s));
    if (geps || gsig)
        LJMD_PHASED(LJMD_PHASE_OTHER, launch_param_grads(part, nb, p->ntypes, geps, gsig, s));
    return LJMD_OK;
}

int ljmd_batch_fm_grad(const double *x, const int32_t *type, const ljmd_batch *b,
                       const ljmd_params *p, const ljmd_nlist *nl, const double *f_target,
                       const double *weight, uint32_t flags, double *f, double *gx, double *geps,
                       double *gsig, void *ws, size_t ws_bytes, void *stream) {
    BatchCtx c;
    int rc = prepare_batch(b, p, &c);
    if (rc) return rc;
    if ((rc = check_batch_nlist(nl, c))) return rc;
    if (nl->mode != LJMD_FULL) return LJMD_ENOTSUP;
    if ((rc = check_batch_built(nl, c))) return rc;
    if (!b->d_offsets || !b->d_boxes) return LJMD_EINVAL;
    if (c.n > 0 && (!x || !f_target || !gx)) return LJMD_EINVAL;
    if (c.n > 0 && p->ntypes > 1 && !type) return LJMD_EINVAL;
    if ((rc = check_batch_ws(ws, ws_bytes, c))) return rc;
    if (c.n <= 0) return LJMD_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    double *g = reinterpret_cast<double *>(w + c.w.xalt);
    double *part = reinterpret_cast<double *>(w + c.bwd_off);
    const int32_t *ty = p->ntypes > 1 ? type : nullptr;
    const FmOut fm{f_target, weight, g};
    if ((rc = batch_plan(b, c, w, s))) return rc;
    if ((rc = batch_forces(x, ty, b, c, nl, (flags & LJMD_PREC_MIXED) != 0, false, f, w, s,
                           nullptr, nullptr, &fm)))
        return rc;
    int64_t nb = 0;
    if (nl->format == LJMD_FMT_TILED)
        LJMD_PHASED(LJMD_PHASE_FORCE,
                    launch_backward_tiled(batch_tile_args(c, nl, w), x, ty, c.n, c.tab,
                                          nl->numneigh, nl->neigh, nl->cap,
                                          (nl->flags & LJMD_NL_SORTED) != 0,
                                          g_gather_lanes.load(), g, gx, part, &nb, s));
    else
        LJMD_PHASED(LJMD_PHASE_FORCE,
                    launch_backward_batch(x, ty, c.n, batch_view(b, c, w), c.tab, nl->numneigh,
                                          nl->neigh, nl->cap, g, gx, part, &nb, s));
    if (geps || gsig)
        LJMD_PHASED(LJMD_PHASE_OTHER, launch_param_grads(part, nb, p->ntypes, geps, gsig, s));
    return LJMD_OK;
}

int ljmd_batch_md_step(double *x, double *v, double *f, int32_t *type, int32_t *id,
                       const ljmd_batch *b, const ljmd_params *p, ljmd_nlist *nl, double dt,
                       int64_t step0, int64_t nsteps, int32_t rebuild_every, int32_t thermo_every,
                       uint32_t flags, double *thermo, void *ws, size_t ws_bytes, void *stream) {
    BatchCtx c;
    int rc = prepare_batch(b, p, &c);
    if (rc) return rc;
    if ((rc = check_batch_nlist(nl, c))) return rc;
    if (!b->d_offsets || !b->d_boxes) return LJMD_EINVAL;
    if (!std::isfinite(dt) || dt <= 0.0) return LJMD_EINVAL;
    if (nsteps < 0 || rebuild_every < 1 || thermo_every < 0 || step0 < 0) return LJMD_EINVAL;
    if (c.n > 0 && (!x || !v || !f)) return LJMD_EINVAL;
    if (c.n > 0 && p->ntypes > 1 && !type) return LJMD_EINVAL;
    if (thermo_every > 0 && !thermo) return LJMD_EINVAL;
    if (!(flags & LJMD_SETUP) && (rc = check_batch_built(nl, c))) return rc;
    double dtf[LJMD_MAX_TYPES] = {0, 0, 0, 0};
    for (int t = 0; t < p->ntypes; ++t) {
        if (!finite_pos(p->mass[t])) return LJMD_EINVAL;
        dtf[t] = 0.5 * dt / p->mass[t];
    }
    if ((rc = check_batch_ws(ws, ws_bytes, c))) return rc;

    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    int32_t *ty = p->ntypes > 1 ? type : nullptr;
    const bool sort = (flags & LJMD_SORT) != 0;
    const int mixed = (flags & LJMD_PREC_MIXED) != 0;
    const double half_skin = 0.5 * p->skin;
    const double *eva = reinterpret_cast<const double *>(w + c.ev_off);
    int64_t row = 0, nbk = 0;
    const int64_t row_len = 9 * (int64_t)c.nrep;

    auto overflowed = [&](bool *out) -> int {
        int32_t st_host[LJMD_STATUS_WORDS];
        LJMD_TRY(hipMemcpyAsync(st_host, nl->status, sizeof(st_host), hipMemcpyDeviceToHost, s));
        LJMD_TRY(hipStreamSynchronize(s));
        *out = st_host[LJMD_ST_OVERFLOW] != 0;
        return LJMD_OK;
    };
    // thermo rows of all systems from the per-atom energy/virial halves and
    // the current (full-step) velocities
    auto thermo_row = [&](int64_t g) -> int {
        LJMD_PHASED(LJMD_PHASE_OTHER,
                    launch_batch_thermo(batch_view(b, c, w), v, ty, p->mass, p->ntypes, eva, c.n,
                                        g, thermo + row_len * row, nullptr, s));
        ++row;
        return LJMD_OK;
    };
    bool ovf = false;
    LJMD_PHASED(LJMD_PHASE_OTHER, launch_set_i32(nl->status, LJMD_STATUS_WORDS, 0, s));
    if ((rc = batch_plan(b, c, w, s))) return rc;
    if (flags & LJMD_SETUP) {
        const bool th = thermo_every > 0 && step0 % thermo_every == 0;
        if ((rc = batch_build(x, ty, b, c, nl, w, s, sort, v, ty, id))) return rc;
        if (flags & LJMD_SYNC_CHECK) {
            if ((rc = overflowed(&ovf))) return rc;
            if (ovf) return LJMD_ENEIGH_OVERFLOW;
        }
        if ((rc = batch_forces(x, ty, b, c, nl, mixed, th, f, w, s))) return rc;
        if (th && (rc = thermo_row(step0))) return rc;
    }
    if (nsteps == 0) return LJMD_OK;
    // With a tiled list the gather applies the velocity-Verlet updates as
    // each atom's force is done (as for one system): mode 2 drifts into the
    // other of two position buffers, mode 1 (thermo steps, whose kinetic
    // energy needs the full-step velocities) only kicks, and the row and the
    // next half kick and drift follow.  The last positions are copied back
    // to x if they ended in the workspace copy; when the buffers change an
    // odd number of times (at every mode-2 step), the first drift already
    // goes to the workspace copy and the last positions land in x.
    const bool fuse = fusable(nl) && !(flags & LJMD_SEPARATE_KICK);
    double *xc = x;
    double *xo = reinterpret_cast<double *>(w + c.w.xalt);
    if (fuse) {
        // steps 1 .. nsteps - 1 that are not thermo steps
        int64_t swaps = nsteps - 1;
        if (thermo_every > 0) swaps -= (step0 + nsteps - 1) / thermo_every - step0 / thermo_every;
        if (swaps % 2 == 1) std::swap(xc, xo);
    }
    LJMD_PHASED(LJMD_PHASE_INTEGRATE,
                launch_kick_drift(x, v, f, ty, c.n, dtf, p->ntypes, dt, s, xc));
    auto copy_back = [&]() -> int {
        if (xc != x)
            LJMD_TRY(hipMemcpyAsync(x, xc, sizeof(double) * 3 * c.n, hipMemcpyDeviceToDevice, s));
        return LJMD_OK;
    };
    for (int64_t st = 1; st <= nsteps; ++st) {
        const int64_t g = step0 + st;
        if (g % rebuild_every == 0) {
            // the binning first checks the displacements since the last build
            if ((rc = batch_build(xc, ty, b, c, nl, w, s, sort, v, ty, id,
                                  half_skin * half_skin)))
                return rc;
            if (flags & LJMD_SYNC_CHECK) {
                if ((rc = overflowed(&ovf))) {
                    (void)copy_back();
                    return rc;
                }
                if (ovf) {
                    if ((rc = copy_back())) return rc;
                    return LJMD_ENEIGH_OVERFLOW;
                }
            }
        }
        const bool th = thermo_every > 0 && g % thermo_every == 0;
        if (fuse) {
            Kick k;
            k.v = v;
            k.xnext = xo;
            k.status = nl->status;
            for (int t = 0; t < kMaxTypes; ++t) {
                k.h[t] = t < p->ntypes ? dtf[t] : 0.0;
                k.mass[t] = t < p->ntypes ? p->mass[t] : 0.0;
            }
            k.dt = dt;
            k.mode = (th || st == nsteps) ? 1 : 2;
            if ((rc = batch_forces(xc, ty, b, c, nl, mixed, th, f, w, s, nullptr, &k))) return rc;
            if (k.mode == 2) {
                std::swap(xc, xo);
                continue;
            }
            if (th && (rc = thermo_row(g))) return rc;
            if (st < nsteps)
                LJMD_PHASED(LJMD_PHASE_INTEGRATE,
                            launch_kick_drift(xc, v, f, ty, c.n, dtf, p->ntypes, dt, s));
            continue;
        }
        if ((rc = batch_forces(xc, ty, b, c, nl, mixed, th, f, w, s))) return rc;
        if (th) {
            // second half kick alone, the row, then the next half kick and
            // drift (the same two fmas as the fused kernel)
            LJMD_PHASED(LJMD_PHASE_INTEGRATE,
                        launch_kick(xc, v, f, ty, c.n, dtf, p->mass, p->ntypes, dt, 0, 0, nullptr,
                                    &nbk, nl->status, s));
            if ((rc = thermo_row(g))) return rc;
            if (st < nsteps)
                LJMD_PHASED(LJMD_PHASE_INTEGRATE,
                            launch_kick_drift(xc, v, f, ty, c.n, dtf, p->ntypes, dt, s));
        } else {
            LJMD_PHASED(LJMD_PHASE_INTEGRATE,
                        launch_kick(xc, v, f, ty, c.n, dtf, p->mass, p->ntypes, dt, st < nsteps, 0,
                                    nullptr, &nbk, nl->status, s));
        }
    }
    return copy_back();
}

int ljmd_batch_set_tuning(const ljmd_batch *b, const ljmd_params *p, uint32_t flags,
                          const ljmd_batch_tuning *t) {
    BatchCtx c;
    int rc = prepare_batch(b, p, &c);
    if (rc) return rc;
    const int mixed = (flags & LJMD_PREC_MIXED) != 0;
    if (t && !tuning_valid(*t)) return LJMD_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int fmt : {LJMD_FMT_GLOBAL, LJMD_FMT_TILED}) {
        if (!t) {
            g_tune.erase(tune_key(c, mixed, fmt));
        } else {
            ljmd_batch_tuning v = *t;
            v.tile_atoms = c.tile_atoms;  // the tiling is the batch's (and its list's)
            g_tune[tune_key(c, mixed, fmt)] = v;
        }
    }
    return LJMD_OK;
}

int ljmd_batch_autotune(double *x, const int32_t *type, const ljmd_batch *b,
                        const ljmd_params *p, ljmd_nlist *nl, uint32_t flags, double *f,
                        void *ws, size_t ws_bytes, void *stream, ljmd_batch_tuning *best) {
    BatchCtx c;
    int rc = prepare_batch(b, p, &c);
    if (rc) return rc;
    if ((rc = check_batch_nlist(nl, c))) return rc;
    if ((rc = check_batch_built(nl, c))) return rc;
    if (!b->d_offsets || !b->d_boxes) return LJMD_EINVAL;
    if (c.n > 0 && (!x || !f)) return LJMD_EINVAL;
    if (c.n > 0 && p->ntypes > 1 && !type) return LJMD_EINVAL;
    if ((rc = check_batch_ws(ws, ws_bytes, c))) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    const int mixed = (flags & LJMD_PREC_MIXED) != 0;
    const int32_t *ty = p->ntypes > 1 ? type : nullptr;
    const bool tiled = nl->format == LJMD_FMT_TILED;
    // the tile target is searched only on a tiled list, and only targets
    // whose workspace and list aux fit the caller's buffers are tried
    const bool search_tiles = tiled && (flags & LJMD_TUNE_TILES) != 0;
    const bool was_sorted = (nl->flags & LJMD_NL_SORTED) != 0;
    std::vector<int> targets;
    if (search_tiles) {
        for (int t : {150, 200, 300, 450, 600}) targets.push_back(t);
    } else {
        targets.push_back(c.tile_atoms);
    }
    hipEvent_t e0, e1;
    LJMD_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return LJMD_EHIP;
    }
    // time `fn` (enqueueing work on s) reps times, the first discarded, and
    // keep the fastest of the others: the candidates differ by a few per
    // cent, about as much as single runs of one of them
    auto timed = [&](int reps, auto fn, float *best_ms) {
        float fastest = 0.0f;
        for (int rep = 0; rep < reps && rc == LJMD_OK; ++rep) {
            if (hipEventRecord(e0, s) != hipSuccess) rc = LJMD_EHIP;
            if (!rc) rc = fn();
            if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = LJMD_EHIP;
            if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = LJMD_EHIP;
            float ms = 0.0f;
            if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = LJMD_EHIP;
            if (rep == 1 || (rep > 1 && ms < fastest)) fastest = ms;
            if (reps == 1) fastest = ms;
        }
        *best_ms = fastest;
    };
    // (re)build nl for batch `bt`
    auto rebuild = [&](const ljmd_batch &bt, const BatchCtx &ct) -> int {
        int r = batch_plan(&bt, ct, w, s);
        if (!r) r = batch_build(x, ty, &bt, ct, nl, w, s);
        return r;
    };
    // after a rebuild: keep the caller's sorted mark when the build left
    // every atom at its own place (the atoms were already in cell order)
    auto mark_sorted = [&](const BatchCtx &ct) -> int {
        if (!was_sorted || ct.n <= 0) return LJMD_OK;
        int32_t *flag = reinterpret_cast<int32_t *>(w + ct.w.tmp);
        const char *aux = static_cast<const char *>(nl->aux);
        const int32_t *perm = reinterpret_cast<const int32_t *>(aux + ct.aux.perm);
        int32_t moved = 1;
        LJMD_TRY(launch_zero_i32(flag, 1, s));
        LJMD_TRY(launch_perm_identity(perm, ct.n, flag, s));
        LJMD_TRY(hipMemcpyAsync(&moved, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        LJMD_TRY(hipStreamSynchronize(s));
        if (!moved) nl->flags |= LJMD_NL_SORTED;
        return LJMD_OK;
    };
    float best_cost = 1e30f;
    ljmd_batch_tuning pick{1, 256, 0, c.tile_atoms};
    // the variants of one tiling: lanes per atom and persistence (512-lane
    // workgroups, one per tile or a persistent grid walking the tiles), and
    // on a global list the workgroup size; lanes 0 (per tile) on tiled lists
    const int lpas[4] = {1, 2, 4, 0}, blocks[2] = {128, 256}, pers[3] = {0, 4, 8};
    for (int target : targets) {
        if (rc) break;
        ljmd_batch bt = *b;
        bt.tile_atoms = target;
        BatchCtx ct;
        if (prepare_batch(&bt, p, &ct) != LJMD_OK) continue;
        if (ct.total > ws_bytes || ct.aux.total > nl->aux_bytes) continue;
        float build_ms = 0.0f, bwd_ms = 0.0f;
        if (search_tiles) {
            timed(3, [&]() { return rebuild(bt, ct); }, &build_ms);
            if (!rc) rc = mark_sorted(ct);
        }
        if (rc) break;
        if ((rc = batch_plan(&bt, ct, w, s))) break;
        float fwd_ms = 1e30f;
        ljmd_batch_tuning local{1, 256, 0, target};
        for (int li = 0; li < (tiled ? 4 : 3) && rc == LJMD_OK; ++li) {
            for (int bi = tiled ? 1 : 0; bi < 2 && rc == LJMD_OK; ++bi) {
                for (int pi = 0; pi < 3 && rc == LJMD_OK; ++pi) {
                    const ljmd_batch_tuning t{lpas[li], blocks[bi], pers[pi], target};
                    float ms = 0.0f;
                    timed(6, [&]() { return batch_forces(x, ty, &bt, ct, nl, mixed, false, f, w,
                                                         s, &t); }, &ms);
                    if (!rc && ms < fwd_ms) {
                        fwd_ms = ms;
                        local = t;
                    }
                }
            }
        }
        if (rc) break;
        if (search_tiles && !(flags & LJMD_TUNE_MD)) {
            // the FP64 adjoint over this tiling (upstream gradient: the forces
            // just computed; result into the workspace's spare vector)
            double *gx = reinterpret_cast<double *>(w + ct.w.xalt);
            double *part = reinterpret_cast<double *>(w + ct.bwd_off);
            timed(5, [&]() {
                int64_t nb = 0;
                LJMD_TRY(launch_backward_tiled(batch_tile_args(ct, nl, w), x, ty, ct.n, ct.tab,
                                               nl->numneigh, nl->neigh, nl->cap,
                                               (nl->flags & LJMD_NL_SORTED) != 0,
                                               g_gather_lanes.load(), f, gx, part, &nb, s));
                return LJMD_OK;
            }, &bwd_ms);
            if (rc) break;
        }
        // cost: the force evaluation, plus with the tile search the build
        // amortized over a 20-step rebuild interval and, unless tuning for
        // the MD step (LJMD_TUNE_MD), the adjoint
        const float cost = fwd_ms + bwd_ms + build_ms / 20.0f;
        if (cost < best_cost) {
            best_cost = cost;
            pick = local;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    if (search_tiles) {
        // leave the list built for the chosen tiling
        ljmd_batch bt = *b;
        bt.tile_atoms = pick.tile_atoms;
        BatchCtx ct;
        if ((rc = prepare_batch(&bt, p, &ct))) return rc;
        if ((rc = rebuild(bt, ct))) return rc;
        if ((rc = mark_sorted(ct))) return rc;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[tune_key(ct, mixed, nl->format)] = pick;
    } else {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[tune_key(c, mixed, nl->format)] = pick;
    }
    if (best) *best = pick;
    return LJMD_OK;
}

int ljmd_get_status(const ljmd_nlist *nl, int32_t *out, void *stream) {
    if (!nl || !nl->status || !out) return LJMD_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    LJMD_TRY(hipMemcpyAsync(out, nl->status, sizeof(int32_t) * LJMD_STATUS_WORDS,
                            hipMemcpyDeviceToHost, s));
    LJMD_TRY(hipStreamSynchronize(s));
    return LJMD_OK;
}

const char *ljmd_strerror(int code) {
    switch (code) {
        case LJMD_OK: return "success";
        case LJMD_EINVAL: return "invalid argument";
        case LJMD_EBOX: return "box length shorter than twice the largest neighbor cutoff";
        case LJMD_EWORKSPACE: return "workspace smaller than ljmd_workspace_bytes()";
        case LJMD_ENEIGH_OVERFLOW: return "neighbor list capacity exceeded";
        case LJMD_ENOTSUP: return "unsupported combination of arguments";
        case LJMD_EHIP: return "HIP runtime error (see ljmd_last_hip_error)";
        case LJMD_ESCRATCH:
            return "problem needs more adjoint blocks than the static scratch of "
                   "ljmd_lj_backward_noalloc holds (LJMD_NOALLOC_MAX_BLOCKS)";
        default: return "unknown error code";
    }
}

const char *ljmd_last_hip_error(void) { return g_last_hip_error.c_str(); }

int ljmd_set_gather_lanes(int lanes) {
    if (lanes != 0 && lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8) return LJMD_EINVAL;
    g_gather_lanes.store(lanes);
    return LJMD_OK;
}

int ljmd_get_gather_lanes(void) { return g_gather_lanes.load(); }

int ljmd_nl_gather_lanes(const ljmd_nlist *nl, const ljmd_box *box, const ljmd_params *p) {
    if (!nl) return LJMD_EINVAL;
    Ctx c;
    int rc = prepare(nl->n, box, p, &c);
    if (rc) return rc;
    if ((rc = check_built(nl, c))) return rc;
    if (nl->format != LJMD_FMT_TILED) return 1;
    return list_lanes(c, nl);
}

int ljmd_profile_enable(int on) {
    g_prof.on = on != 0;
    return LJMD_OK;
}

int ljmd_profile_read(double *ms, int64_t *launches) {
    if (!ms || !launches) return LJMD_EINVAL;
    for (int k = 0; k < LJMD_PHASES; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    int rc = LJMD_OK;
    for (const Mark &m : g_prof.marks) {
        float t = 0.0f;
        hipError_t e = hipEventSynchronize(m.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, m.a, m.b);
        if (e != hipSuccess) {
            g_last_hip_error = hipGetErrorString(e);
            rc = LJMD_EHIP;
        } else if (m.phase >= 0 && m.phase < LJMD_PHASES) {
            ms[m.phase] += t;
            launches[m.phase] += 1;
        }
        g_prof.pool.push_back(m.a);
        g_prof.pool.push_back(m.b);
    }
    g_prof.marks.clear();
    return rc;
}

}  // extern "C"
