/*
 * ljref.c -- plain serial FP64 CPU oracle for the Lennard-Jones MD hot path.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library.  It
 * shares no code with the HIP library; it is compiled with gcc and
 * -ffp-contract=off so that the only fused multiply-adds are the explicit
 * fma() calls below.
 *
 * Every routine follows the plain definition of what the hot path computes,
 * from arXiv:2508.13523 (LAMMPS-KOKKOS):
 *   Sec. 4, Eq. (1)   E = sum_{i<k, r_ik < r_c} 4 eps [(sigma/r)^12 - (sigma/r)^6]
 *   Sec. 4            forces are the pairwise sum of -dU/dr, summed over pairs
 *                     taken from a neighbor list that is rebuilt periodically
 *   Sec. 4.1          full lists hold every pair twice (once per atom), half
 *                     lists hold each pair once (Newton's third law)
 * The velocity-Verlet integrator, the skin and the wrap rule are not in the
 * paper (it only says Newton's second law is integrated, Sec. 1); they follow
 * the readings listed in ljref.h.
 *
 * Parity status: the pair force/energy, the neighbor lists, the virial, the
 * integrator and the adjoint are each pinned by independent checks in the
 * test suite (closed forms, lattice sums, brute force, finite differences).
 */
#include "ljref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* geometry                                                            */
/* ------------------------------------------------------------------ */

/* Wrap one coordinate into [0, L) (branch form, no division). */
static double wrap1(double x, double L)
{
    if (x < 0.0)
        x += L;
    else if (x >= L)
        x -= L;
    if (x == L) /* a tiny negative x plus L can round up to L */
        x = 0.0;
    return x;
}

void ref_wrap(int64_t n, double *x, const double *box)
{
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d)
            x[3 * i + d] = wrap1(x[3 * i + d], box[d]);
}

/* Minimum image of one displacement component, branch form.  Valid while
 * both coordinates lie within half a box of [0, L). */
static double min_image(double d, double L)
{
    const double h = 0.5 * L;
    if (d > h)
        return d - L;
    if (d < -h)
        return d + L;
    return d;
}

/* d = x_i - x_j under the minimum image; returns |d|^2. */
static double pair_disp(const double *x, int64_t i, int64_t j,
                        const double *box, double *d)
{
    d[0] = min_image(x[3 * i + 0] - x[3 * j + 0], box[0]);
    d[1] = min_image(x[3 * i + 1] - x[3 * j + 1], box[1]);
    d[2] = min_image(x[3 * i + 2] - x[3 * j + 2], box[2]);
    return fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0]));
}

/* ------------------------------------------------------------------ */
/* pair enumeration: every unordered pair i<j, or those within `cut`   */
/* ------------------------------------------------------------------ */

typedef void (*pair_fn)(int64_t i, int64_t j, const double *d, double rsq,
                        void *ctx);

/* All n(n-1)/2 pairs, in order i ascending then j ascending. */
static void enum_brute(int64_t n, const double *x, const double *box,
                       pair_fn fn, void *ctx)
{
    double d[3];
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            const double rsq = pair_disp(x, i, j, box, d);
            fn(i, j, d, rsq, ctx);
        }
}

/* Pairs with |d| < cut via a uniform cell grid.  Cells are at least
 * cut*(1+1e-9) wide so that rounding in the binning can never separate two
 * atoms closer than cut by more than one cell.  The 3x3x3 stencil is
 * de-duplicated per dimension, so grids with one or two cells per dimension
 * visit each cell once.  Each unordered pair is visited once: in the cell of
 * the lower index, with the higher index in a stencil cell. */
static void enum_cells(int64_t n, const double *x, const double *box,
                       double cut, pair_fn fn, void *ctx)
{
    int nc[3];
    for (int k = 0; k < 3; ++k) {
        nc[k] = (int)floor(box[k] / (cut * (1.0 + 1e-9)));
        if (nc[k] < 1)
            nc[k] = 1;
    }
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * ncell);
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    for (int64_t c = 0; c < ncell; ++c)
        head[c] = -1;
    for (int64_t i = n - 1; i >= 0; --i) {
        int cc[3];
        for (int k = 0; k < 3; ++k) {
            const double w = wrap1(x[3 * i + k], box[k]);
            int c = (int)(w * nc[k] / box[k]);
            if (c >= nc[k])
                c = nc[k] - 1;
            if (c < 0)
                c = 0;
            cc[k] = c;
        }
        cell[i] = ((int64_t)cc[2] * nc[1] + cc[1]) * nc[0] + cc[0];
        next[i] = head[cell[i]];
        head[cell[i]] = i;
    }
    const double cut2 = cut * cut;
    double d[3];
    for (int64_t c = 0; c < ncell; ++c) {
        const int cx = (int)(c % nc[0]);
        const int cy = (int)((c / nc[0]) % nc[1]);
        const int cz = (int)(c / ((int64_t)nc[0] * nc[1]));
        int nb[3][3], nnb[3];
        const int cc[3] = {cx, cy, cz};
        for (int k = 0; k < 3; ++k) {
            nnb[k] = 0;
            for (int o = -1; o <= 1; ++o) {
                const int v = ((cc[k] + o) % nc[k] + nc[k]) % nc[k];
                int seen = 0;
                for (int q = 0; q < nnb[k]; ++q)
                    if (nb[k][q] == v)
                        seen = 1;
                if (!seen)
                    nb[k][nnb[k]++] = v;
            }
        }
        for (int a = 0; a < nnb[2]; ++a)
            for (int b = 0; b < nnb[1]; ++b)
                for (int e = 0; e < nnb[0]; ++e) {
                    const int64_t c2 =
                        ((int64_t)nb[2][a] * nc[1] + nb[1][b]) * nc[0] +
                        nb[0][e];
                    for (int64_t i = head[c]; i >= 0; i = next[i])
                        for (int64_t j = head[c2]; j >= 0; j = next[j]) {
                            if (j <= i)
                                continue;
                            const double rsq = pair_disp(x, i, j, box, d);
                            if (rsq < cut2)
                                fn(i, j, d, rsq, ctx);
                        }
                }
    }
    free(head);
    free(next);
    free(cell);
}

/* ------------------------------------------------------------------ */
/* neighbor lists (Sec. 4; full/half: Sec. 4.1)                        */
/* ------------------------------------------------------------------ */

typedef struct {
    const int32_t *type;
    int32_t ntypes;
    const double *rnb2; /* (rc_ij + skin)^2 */
    int32_t half;
    int64_t *counts;
    const int64_t *offsets;
    int32_t *idx;
    int64_t *cursor;
    int64_t total;
} nl_ctx;

static void nl_pair(int64_t i, int64_t j, const double *d, double rsq,
                    void *vctx)
{
    (void)d;
    nl_ctx *c = (nl_ctx *)vctx;
    const int32_t ti = c->type[i], tj = c->type[j];
    if (!(rsq < c->rnb2[ti * c->ntypes + tj]))
        return;
    /* row i gets j; a full list also gives row j the entry i */
    c->counts[i]++;
    c->total++;
    if (c->idx)
        c->idx[c->offsets[i] + c->cursor[i]++] = (int32_t)j;
    if (!c->half) {
        c->counts[j]++;
        c->total++;
        if (c->idx)
            c->idx[c->offsets[j] + c->cursor[j]++] = (int32_t)i;
    }
}

static int cmp_i32(const void *a, const void *b)
{
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static double *make_rnb2(int32_t ntypes, const double *rc, double skin,
                         double *maxcut)
{
    double *t = (double *)malloc(sizeof(double) * ntypes * ntypes);
    *maxcut = 0.0;
    for (int k = 0; k < ntypes * ntypes; ++k) {
        const double r = rc[k] + skin;
        t[k] = r * r;
        if (r > *maxcut)
            *maxcut = r;
    }
    return t;
}

/* Two-call protocol: with idx == NULL, fill counts[n] and return the total;
 * with idx != NULL (and offsets from the caller's prefix sum of counts),
 * also fill idx.  Rows come out sorted ascending.  Positions are wrapped
 * into the box (on a copy) before the distance test. */
static int64_t nl_common(int use_cells, int64_t n, const double *x,
                         const int32_t *type, const double *box,
                         int32_t ntypes, const double *rc, double skin,
                         int32_t half, int64_t *counts,
                         const int64_t *offsets, int32_t *idx)
{
    double *xw = (double *)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    memcpy(xw, x, sizeof(double) * 3 * n);
    ref_wrap(n, xw, box);
    double maxcut;
    double *rnb2 = make_rnb2(ntypes, rc, skin, &maxcut);
    nl_ctx c = {type, ntypes, rnb2, half, counts, offsets, idx, NULL, 0};
    memset(counts, 0, sizeof(int64_t) * n);
    if (idx) {
        c.cursor = (int64_t *)calloc(n > 0 ? n : 1, sizeof(int64_t));
    }
    if (use_cells)
        enum_cells(n, xw, box, maxcut, nl_pair, &c);
    else
        enum_brute(n, xw, box, nl_pair, &c);
    if (idx) {
        for (int64_t i = 0; i < n; ++i)
            qsort(idx + offsets[i], (size_t)counts[i], sizeof(int32_t),
                  cmp_i32);
        free(c.cursor);
    }
    free(rnb2);
    free(xw);
    return c.total;
}

int64_t ref_nl_brute(int64_t n, const double *x, const int32_t *type,
                     const double *box, int32_t ntypes, const double *rc,
                     double skin, int32_t half, int64_t *counts,
                     const int64_t *offsets, int32_t *idx)
{
    return nl_common(0, n, x, type, box, ntypes, rc, skin, half, counts,
                     offsets, idx);
}

int64_t ref_nl_cells(int64_t n, const double *x, const int32_t *type,
                     const double *box, int32_t ntypes, const double *rc,
                     double skin, int32_t half, int64_t *counts,
                     const int64_t *offsets, int32_t *idx)
{
    return nl_common(1, n, x, type, box, ntypes, rc, skin, half, counts,
                     offsets, idx);
}

/* Full-list rows of selected atoms only, by brute force over all j (O(n)
 * per row); for spot checks on systems too large for a whole list. */
int64_t ref_nl_rows(int64_t n, const double *x, const int32_t *type,
                    const double *box, int32_t ntypes, const double *rc,
                    double skin, int64_t nrows, const int64_t *rows,
                    int64_t *counts, const int64_t *offsets, int32_t *idx)
{
    double maxcut;
    double *rnb2 = make_rnb2(ntypes, rc, skin, &maxcut);
    int64_t total = 0;
    double d[3];
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t i = rows[r];
        double xi[3];
        for (int k = 0; k < 3; ++k)
            xi[k] = wrap1(x[3 * i + k], box[k]);
        int64_t cnt = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            for (int k = 0; k < 3; ++k)
                d[k] = min_image(xi[k] - wrap1(x[3 * j + k], box[k]), box[k]);
            const double rsq = fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0]));
            if (rsq < rnb2[type[i] * ntypes + type[j]]) {
                if (idx)
                    idx[offsets[r] + cnt] = (int32_t)j;
                cnt++;
            }
        }
        counts[r] = cnt;
        total += cnt;
    }
    free(rnb2);
    return total;
}

/* ------------------------------------------------------------------ */
/* forces, energy, virial (Sec. 4, Eq. (1))                            */
/* ------------------------------------------------------------------ */

typedef struct {
    const int32_t *type;
    int32_t ntypes;
    const double *eps, *sigma;
    double *rc2;
    double *f;
    double ev[7];
} force_ctx;

/* Textbook 12-6 pair: with s2 = sigma^2/r^2 and s6 = s2^3,
 *   U(r)   = 4 eps (s6^2 - s6)
 *   -dU/dr / r = 24 eps (2 s6^2 - s6) / r^2      (= fpair)
 * so the force on i from j is fpair * (x_i - x_j). */
static void force_pair(int64_t i, int64_t j, const double *d, double rsq,
                       void *vctx)
{
    force_ctx *c = (force_ctx *)vctx;
    const int k = c->type[i] * c->ntypes + c->type[j];
    if (!(rsq < c->rc2[k]))
        return;
    const double e = c->eps[k], s = c->sigma[k];
    const double s2 = (s * s) / rsq;
    const double s6 = s2 * s2 * s2;
    const double u = 4.0 * e * (s6 * s6 - s6);
    const double fpair = 24.0 * e * (2.0 * s6 * s6 - s6) / rsq;
    for (int a = 0; a < 3; ++a) {
        c->f[3 * i + a] += fpair * d[a];
        c->f[3 * j + a] -= fpair * d[a];
    }
    c->ev[0] += u;
    c->ev[1] += d[0] * d[0] * fpair;
    c->ev[2] += d[1] * d[1] * fpair;
    c->ev[3] += d[2] * d[2] * fpair;
    c->ev[4] += d[0] * d[1] * fpair;
    c->ev[5] += d[0] * d[2] * fpair;
    c->ev[6] += d[1] * d[2] * fpair;
}

static double *make_rc2(int32_t ntypes, const double *rc, double *maxcut)
{
    double *t = (double *)malloc(sizeof(double) * ntypes * ntypes);
    *maxcut = 0.0;
    for (int k = 0; k < ntypes * ntypes; ++k) {
        t[k] = rc[k] * rc[k];
        if (rc[k] > *maxcut)
            *maxcut = rc[k];
    }
    return t;
}

static void forces_common(int use_cells, int64_t n, const double *x,
                          const int32_t *type, const double *box,
                          int32_t ntypes, const double *eps,
                          const double *sigma, const double *rc, double *f,
                          double *ev)
{
    double maxcut;
    force_ctx c;
    c.type = type;
    c.ntypes = ntypes;
    c.eps = eps;
    c.sigma = sigma;
    c.rc2 = make_rc2(ntypes, rc, &maxcut);
    c.f = f;
    memset(c.ev, 0, sizeof(c.ev));
    memset(f, 0, sizeof(double) * 3 * n);
    if (use_cells)
        enum_cells(n, x, box, maxcut, force_pair, &c);
    else
        enum_brute(n, x, box, force_pair, &c);
    if (ev)
        memcpy(ev, c.ev, sizeof(c.ev));
    free(c.rc2);
}

void ref_forces_brute(int64_t n, const double *x, const int32_t *type,
                      const double *box, int32_t ntypes, const double *eps,
                      const double *sigma, const double *rc, double *f,
                      double *ev)
{
    forces_common(0, n, x, type, box, ntypes, eps, sigma, rc, f, ev);
}

void ref_forces_cells(int64_t n, const double *x, const int32_t *type,
                      const double *box, int32_t ntypes, const double *eps,
                      const double *sigma, const double *rc, double *f,
                      double *ev)
{
    forces_common(1, n, x, type, box, ntypes, eps, sigma, rc, f, ev);
}

/* Force on selected atoms only, by brute force over all j (O(n) per row). */
void ref_force_rows(int64_t n, const double *x, const int32_t *type,
                    const double *box, int32_t ntypes, const double *eps,
                    const double *sigma, const double *rc, int64_t nrows,
                    const int64_t *rows, double *frows)
{
    double maxcut;
    double *rc2 = make_rc2(ntypes, rc, &maxcut);
    double d[3];
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t i = rows[r];
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            const double rsq = pair_disp(x, i, j, box, d);
            const int k = type[i] * ntypes + type[j];
            if (!(rsq < rc2[k]))
                continue;
            const double e = eps[k], s = sigma[k];
            const double s2 = (s * s) / rsq;
            const double s6 = s2 * s2 * s2;
            const double fpair = 24.0 * e * (2.0 * s6 * s6 - s6) / rsq;
            for (int a = 0; a < 3; ++a)
                acc[a] += fpair * d[a];
        }
        for (int a = 0; a < 3; ++a)
            frows[3 * r + a] = acc[a];
    }
    free(rc2);
}

/* ------------------------------------------------------------------ */
/* adjoint of the force map                                            */
/* ------------------------------------------------------------------ */
/*
 * Given g_i = dL/dF_i, the pair (i,j) adds gamma(r) d to F_i and -gamma(r) d
 * to F_j, with d = x_i - x_j and gamma = fpair = 24 eps (2 s6^2 - s6)/r^2.
 * Differentiating gamma(r) d with respect to d:
 *   dL/dx_i += gamma (g_i - g_j) + (gamma'(r)/r) (d . (g_i - g_j)) d
 *   dL/dx_j -= the same,
 *   gamma'(r)/r = -24 eps (28 s6^2 - 8 s6) / r^4.
 * Parameter derivatives of gamma at fixed r (cutoff held fixed):
 *   d gamma / d eps   = gamma / eps
 *   d gamma / d sigma = 24 eps (24 s6^2 - 6 s6) / (sigma r^2)
 * and dL/dtheta += (d gamma/d theta) (d . (g_i - g_j)).
 * Table convention: for a pair of unlike types the contribution is split
 * evenly between entries [a][b] and [b][a], so the table gradient is
 * symmetric and the gradient of the shared parameter is their sum.
 */
typedef struct {
    const int32_t *type;
    int32_t ntypes;
    const double *eps, *sigma;
    double *rc2;
    const double *g;
    double *gx, *geps, *gsig;
} bwd_ctx;

static void bwd_pair(int64_t i, int64_t j, const double *d, double rsq,
                     void *vctx)
{
    bwd_ctx *c = (bwd_ctx *)vctx;
    const int32_t ti = c->type[i], tj = c->type[j];
    const int k = ti * c->ntypes + tj;
    if (!(rsq < c->rc2[k]))
        return;
    const double e = c->eps[k], s = c->sigma[k];
    const double s2 = (s * s) / rsq;
    const double s6 = s2 * s2 * s2;
    const double gam = 24.0 * e * (2.0 * s6 * s6 - s6) / rsq;
    const double dgam_r = -24.0 * e * (28.0 * s6 * s6 - 8.0 * s6) / (rsq * rsq);
    double gd[3];
    for (int a = 0; a < 3; ++a)
        gd[a] = c->g[3 * i + a] - c->g[3 * j + a];
    const double dot = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
    for (int a = 0; a < 3; ++a) {
        const double t = gam * gd[a] + dgam_r * dot * d[a];
        c->gx[3 * i + a] += t;
        c->gx[3 * j + a] -= t;
    }
    const double de = gam / e * dot;
    const double ds = 24.0 * e * (24.0 * s6 * s6 - 6.0 * s6) / (s * rsq) * dot;
    if (ti == tj) {
        c->geps[k] += de;
        c->gsig[k] += ds;
    } else {
        const int kt = tj * c->ntypes + ti;
        c->geps[k] += 0.5 * de;
        c->geps[kt] += 0.5 * de;
        c->gsig[k] += 0.5 * ds;
        c->gsig[kt] += 0.5 * ds;
    }
}

static void bwd_common(int use_cells, int64_t n, const double *x,
                       const int32_t *type, const double *box, int32_t ntypes,
                       const double *eps, const double *sigma,
                       const double *rc, const double *g, double *gx,
                       double *geps, double *gsig)
{
    double maxcut;
    bwd_ctx c;
    c.type = type;
    c.ntypes = ntypes;
    c.eps = eps;
    c.sigma = sigma;
    c.rc2 = make_rc2(ntypes, rc, &maxcut);
    c.g = g;
    c.gx = gx;
    c.geps = geps;
    c.gsig = gsig;
    memset(gx, 0, sizeof(double) * 3 * n);
    memset(geps, 0, sizeof(double) * ntypes * ntypes);
    memset(gsig, 0, sizeof(double) * ntypes * ntypes);
    if (use_cells)
        enum_cells(n, x, box, maxcut, bwd_pair, &c);
    else
        enum_brute(n, x, box, bwd_pair, &c);
    free(c.rc2);
}

void ref_backward_brute(int64_t n, const double *x, const int32_t *type,
                        const double *box, int32_t ntypes, const double *eps,
                        const double *sigma, const double *rc, const double *g,
                        double *gx, double *geps, double *gsig)
{
    bwd_common(0, n, x, type, box, ntypes, eps, sigma, rc, g, gx, geps, gsig);
}

void ref_backward_cells(int64_t n, const double *x, const int32_t *type,
                        const double *box, int32_t ntypes, const double *eps,
                        const double *sigma, const double *rc, const double *g,
                        double *gx, double *geps, double *gsig)
{
    bwd_common(1, n, x, type, box, ntypes, eps, sigma, rc, g, gx, geps, gsig);
}

/* ------------------------------------------------------------------ */
/* velocity Verlet                                                     */
/* ------------------------------------------------------------------ */

double ref_kinetic(int64_t n, const double *v, const int32_t *type,
                   const double *mass)
{
    double ke = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double m = mass[type[i]];
        for (int a = 0; a < 3; ++a)
            ke += 0.5 * m * v[3 * i + a] * v[3 * i + a];
    }
    return ke;
}

static void thermo_row(double *row, int64_t g, const double *ev, double ke)
{
    row[0] = (double)g;
    row[1] = ev[0];
    row[2] = ke;
    for (int k = 0; k < 6; ++k)
        row[3 + k] = ev[1 + k];
}

/* ------------------------------------------------------------------ */
/* Verlet pair list: the pair sum of Sec. 4 taken over a list that is  */
/* rebuilt periodically, not over all pairs                            */
/* ------------------------------------------------------------------ */

/* Each stored pair i<j keeps the image chosen at the build (per dimension:
 * 0 none, 1 subtract L, 2 add L), so that between builds the displacement is
 * d = x_i - x_j corrected by that image, whatever the atoms' positions. */
typedef struct {
    int64_t *i, *j;
    int32_t *code;
    int64_t count, capacity;
    const int32_t *type;
    int32_t ntypes;
    const double *rnb2;
    const double *x;
    const double *box;
} vlist;

static void vlist_pair(int64_t i, int64_t j, const double *d, double rsq, void *vctx)
{
    (void)d;
    vlist *l = (vlist *)vctx;
    if (!(rsq < l->rnb2[l->type[i] * l->ntypes + l->type[j]]))
        return;
    if (l->count == l->capacity) {
        l->capacity = l->capacity ? 2 * l->capacity : 1024;
        l->i = (int64_t *)realloc(l->i, sizeof(int64_t) * l->capacity);
        l->j = (int64_t *)realloc(l->j, sizeof(int64_t) * l->capacity);
        l->code = (int32_t *)realloc(l->code, sizeof(int32_t) * l->capacity);
    }
    int32_t code = 0;
    for (int a = 0; a < 3; ++a) {
        const double raw = l->x[3 * i + a] - l->x[3 * j + a];
        const double h = 0.5 * l->box[a];
        if (raw > h)
            code |= 1 << (2 * a);
        else if (raw < -h)
            code |= 2 << (2 * a);
    }
    l->i[l->count] = i;
    l->j[l->count] = j;
    l->code[l->count] = code;
    l->count++;
}

static void vlist_build(vlist *l, int64_t n, const double *x, double maxcut)
{
    l->count = 0;
    l->x = x;
    enum_cells(n, x, l->box, maxcut, vlist_pair, l);
}

static void vlist_forces(const vlist *l, int64_t n, const double *x, const double *eps,
                         const double *sigma, const double *rc2, double *f, double *ev)
{
    memset(f, 0, sizeof(double) * 3 * n);
    for (int k = 0; k < 7; ++k)
        ev[k] = 0.0;
    force_ctx c;
    c.type = l->type;
    c.ntypes = l->ntypes;
    c.eps = eps;
    c.sigma = sigma;
    c.rc2 = (double *)rc2;
    c.f = f;
    memset(c.ev, 0, sizeof(c.ev));
    for (int64_t p = 0; p < l->count; ++p) {
        const int64_t i = l->i[p], j = l->j[p];
        double d[3];
        for (int a = 0; a < 3; ++a) {
            d[a] = x[3 * i + a] - x[3 * j + a];
            const int32_t cd = (l->code[p] >> (2 * a)) & 3;
            if (cd == 1)
                d[a] -= l->box[a];
            else if (cd == 2)
                d[a] += l->box[a];
        }
        const double rsq = fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0]));
        force_pair(i, j, d, rsq, &c);
    }
    memcpy(ev, c.ev, sizeof(c.ev));
}

/* Velocity Verlet, one step:
 *   v += (dt/2m) f;  x += dt v;  [rebuild steps: wrap x, rebuild list];
 *   f = F(x);  v += (dt/2m) f.
 * Step g = step0 + s for s = 1..nsteps.  Positions are wrapped into the box
 * on steps with g % rebuild_every == 0.  With skin >= 0 the forces are the
 * pair sum over a Verlet list of cutoff rc_ij + skin rebuilt on exactly those
 * steps (Sec. 4: the pair sum runs over a list that is built and updated
 * periodically), so a pair that closes in from beyond the list cutoff between
 * builds is missed, as in the method.  With skin < 0 the forces are the exact
 * pair sum at every step.  With `setup`, x is wrapped, the list built and f
 * computed before the first step.  Thermo rows [g, E, KE, Wxx, Wyy, Wzz, Wxy,
 * Wxz, Wyz] are written for every g with g % thermo_every == 0 (g = step0
 * only with setup).  Returns the row count. */
static int64_t md_core(int64_t n, double *x, double *v, double *f,
                       const int32_t *type, const double *box, int32_t ntypes,
                       const double *eps, const double *sigma, const double *rc,
                       const double *mass, double skin, double dt, int64_t step0,
                       int64_t nsteps, int32_t rebuild_every, int32_t thermo_every,
                       int32_t setup, double *thermo, double rescale_t)
{
    double ev[7];
    int64_t rows = 0;
    double *dtf = (double *)malloc(sizeof(double) * ntypes);
    for (int t = 0; t < ntypes; ++t)
        dtf[t] = 0.5 * dt / mass[t];
    const int use_list = skin >= 0.0;
    double maxcut = 0.0, maxrc;
    double *rnb2 = use_list ? make_rnb2(ntypes, rc, skin, &maxcut) : NULL;
    double *rc2 = make_rc2(ntypes, rc, &maxrc);
    vlist l;
    memset(&l, 0, sizeof(l));
    l.type = type;
    l.ntypes = ntypes;
    l.rnb2 = rnb2;
    l.box = box;
#define LJREF_FORCES()                                                       \
    do {                                                                     \
        if (use_list)                                                        \
            vlist_forces(&l, n, x, eps, sigma, rc2, f, ev);                  \
        else                                                                 \
            ref_forces_cells(n, x, type, box, ntypes, eps, sigma, rc, f, ev); \
    } while (0)
    if (setup) {
        ref_wrap(n, x, box);
        if (use_list)
            vlist_build(&l, n, x, maxcut);
        LJREF_FORCES();
        if (thermo_every > 0 && step0 % thermo_every == 0 && thermo)
            thermo_row(thermo + 9 * rows++, step0, ev,
                       ref_kinetic(n, v, type, mass));
    } else if (use_list) {
        vlist_build(&l, n, x, maxcut);
    }
    for (int64_t s = 1; s <= nsteps; ++s) {
        const int64_t g = step0 + s;
        for (int64_t i = 0; i < n; ++i) {
            const double h = dtf[type[i]];
            for (int a = 0; a < 3; ++a) {
                v[3 * i + a] = fma(h, f[3 * i + a], v[3 * i + a]);
                x[3 * i + a] = fma(dt, v[3 * i + a], x[3 * i + a]);
            }
        }
        if (rebuild_every > 0 && g % rebuild_every == 0) {
            ref_wrap(n, x, box);
            if (use_list)
                vlist_build(&l, n, x, maxcut);
        }
        LJREF_FORCES();
        for (int64_t i = 0; i < n; ++i) {
            const double h = dtf[type[i]];
            for (int a = 0; a < 3; ++a)
                v[3 * i + a] = fma(h, f[3 * i + a], v[3 * i + a]);
        }
        if (rescale_t > 0.0 && n > 1) {
            /* velocity rescaling to the kinetic temperature rescale_t
             * (3n - 3 degrees of freedom) */
            const double ke = ref_kinetic(n, v, type, mass);
            if (ke > 0.0) {
                const double s = sqrt(0.5 * (double)(3 * n - 3) * rescale_t / ke);
                for (int64_t i = 0; i < 3 * n; ++i)
                    v[i] *= s;
            }
        }
        if (thermo_every > 0 && g % thermo_every == 0 && thermo)
            thermo_row(thermo + 9 * rows++, g, ev,
                       ref_kinetic(n, v, type, mass));
    }
#undef LJREF_FORCES
    free(l.i);
    free(l.j);
    free(l.code);
    free(rnb2);
    free(rc2);
    free(dtf);
    return rows;
}

int64_t ref_md(int64_t n, double *x, double *v, double *f,
               const int32_t *type, const double *box, int32_t ntypes,
               const double *eps, const double *sigma, const double *rc,
               const double *mass, double skin, double dt, int64_t step0,
               int64_t nsteps, int32_t rebuild_every, int32_t thermo_every,
               int32_t setup, double *thermo)
{
    return md_core(n, x, v, f, type, box, ntypes, eps, sigma, rc, mass, skin, dt, step0,
                   nsteps, rebuild_every, thermo_every, setup, thermo, 0.0);
}

/* ref_md with the velocities rescaled after every step so that the kinetic
 * temperature (3n - 3 degrees of freedom) is exactly temp: the equilibration
 * of a freshly placed liquid (input preparation; not part of the method). */
int64_t ref_md_rescale(int64_t n, double *x, double *v, double *f,
                       const int32_t *type, const double *box, int32_t ntypes,
                       const double *eps, const double *sigma, const double *rc,
                       const double *mass, double skin, double dt, int64_t nsteps,
                       int32_t rebuild_every, double temp)
{
    return md_core(n, x, v, f, type, box, ntypes, eps, sigma, rc, mass, skin, dt, 0,
                   nsteps, rebuild_every, 0, 1, NULL, temp);
}
