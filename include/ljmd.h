/*
 * ljmd.h -- C ABI of the MI355X (gfx950) Lennard-Jones MD hot path.
 *
 * The library computes, on one GPU, the pairwise Lennard-Jones workload of
 * Johansson et al., "LAMMPS-KOKKOS: Performance Portable Molecular Dynamics
 * Across Exascale Architectures" (arXiv:2508.13523):
 *   - a binned Verlet neighbor list, full or half (Sec. 4: the pair sum runs
 *     over a neighbor list that is built and periodically updated; Sec. 4.1:
 *     half lists use Newton's third law, full lists compute each pair twice);
 *   - the 12-6 energy of Sec. 4, Eq. (1), its forces (the pairwise sum of
 *     -dU/dr, Sec. 4) and the virial, over that list;
 *   - a velocity-Verlet step driving both;
 *   - the adjoint of the force map (gradients of a scalar loss of the forces
 *     with respect to positions and the per-type-pair eps/sigma tables).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers (hipMalloc'ed or torch CUDA
 *    tensors) unless marked "host".  The caller owns every buffer; the
 *    library never allocates or frees device memory.
 *  - x, v, f, gF, gx are row-major [n][3] float64 (atom i at offset 3*i).
 *    type is [n] int32 in [0, ntypes); it may be NULL when ntypes == 1.
 *  - The box is periodic and orthorhombic with origin 0: [0, len[d]).
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = default stream)
 *    and runs asynchronously.  No entry point synchronizes the stream except
 *    ljmd_get_status, ljmd_md_step / ljmd_batch_md_step with LJMD_SYNC_CHECK
 *    and ljmd_batch_autotune.
 *  - Return value: LJMD_OK (0) or a negative LJMD_E* code.  All argument
 *    checks run on the host before any work is enqueued, so a rejected call
 *    has no side effect.  LJMD_EHIP reports a HIP runtime failure;
 *    ljmd_strerror() describes every code.
 *  - Cutoffs are strict: a pair interacts when r < rc_ij (Eq. (1)); the
 *    energy is truncated, not shifted.  A pair is a neighbor when
 *    r < rc_ij + skin.  Distances use the minimum image; every box length
 *    must be at least 2 * max(rc_ij + skin) (else LJMD_EBOX).
 *  - Atom counts: 0 <= n < 2^26 (neighbor entries pack a 26-bit atom index
 *    with 6 bits of periodic-image code).  Offsets into the neighbor array
 *    are 64-bit (App. B: table offsets, not indices, outgrow 32 bits).
 */
#ifndef LJMD_H
#define LJMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LJMD_MAX_TYPES 4
#define LJMD_MAX_ATOMS (1LL << 26)
#define LJMD_STATUS_WORDS 4

/* ---- return codes ---- */
#define LJMD_OK 0
#define LJMD_EINVAL (-1)          /* bad argument (NULL pointer, n, table...) */
#define LJMD_EBOX (-2)            /* box shorter than 2 * max neighbor cutoff */
#define LJMD_EWORKSPACE (-3)      /* ws_bytes < ljmd_workspace_bytes(...)     */
#define LJMD_ENEIGH_OVERFLOW (-4) /* an atom has more neighbors than cap      */
#define LJMD_ENOTSUP (-5)         /* valid but unsupported combination        */
#define LJMD_EHIP (-6)            /* HIP runtime error                        */
#define LJMD_ESCRATCH (-7)        /* larger than the static scratch of
                                     ljmd_lj_backward_noalloc                 */

/* ---- flags ---- */
#define LJMD_PREC_FP64 0u          /* all pair arithmetic in FP64            */
#define LJMD_PREC_MIXED (1u << 0)  /* FP64 positions, displacement, r^2 and
                                      cutoff test; FP32 pair terms; FP64
                                      accumulation of f, E and W            */
#define LJMD_EV (1u << 1)          /* also compute energy and virial        */
#define LJMD_SYNC_CHECK (1u << 2)  /* md_step: read the status word after
                                      every rebuild and stop on overflow    */
#define LJMD_SETUP (1u << 3)       /* md_step: build the list and compute f
                                      before the first step                 */
#define LJMD_SORT (1u << 4)        /* md_step: at every build, reorder the
                                      atoms (x, v, type, id) into cell order */
#define LJMD_SEPARATE_KICK (1u << 5) /* md_step: run the velocity-Verlet
                                      updates as kernels of their own even
                                      where the force kernel can apply them
                                      (results are bit-identical)          */

/* ---- neighbor list modes ---- */
#define LJMD_FULL 0 /* every neighbor j of i in row i; forces by gather    */
#define LJMD_HALF 1 /* pair (i,j) only in row min(i,j); forces by scatter  */

/* ---- status words (device int32[LJMD_STATUS_WORDS]) ---- */
#define LJMD_ST_OVERFLOW 0  /* bit 0: some atom had more than cap neighbors;
                               bit 1: a tile's stencil held 65536 atoms or
                               more (tiled format impossible: build again
                               with LJMD_NL_GLOBAL)                       */
#define LJMD_ST_NEED 1      /* largest neighbor count seen                 */
#define LJMD_ST_DANGEROUS 2 /* 1 if an atom moved more than skin/2 between
                               two builds (md_step only)                  */
#define LJMD_ST_NONFINITE 3 /* 1 if a non-finite velocity appeared         */

/* Periodic orthorhombic box (host struct).  Every length must be finite,
 * positive and below 1e9 (else LJMD_EINVAL). */
typedef struct {
    double len[3];
} ljmd_box;

/* Force-field parameters (host struct).  The eps, sigma and rc tables are
 * indexed [type_i][type_j], must be symmetric, and only the leading
 * ntypes x ntypes block is read.  mass[t] is used by md_step only. */
typedef struct {
    int32_t ntypes;
    int32_t reserved;
    double eps[LJMD_MAX_TYPES][LJMD_MAX_TYPES];
    double sigma[LJMD_MAX_TYPES][LJMD_MAX_TYPES];
    double rc[LJMD_MAX_TYPES][LJMD_MAX_TYPES];
    double skin;
    double mass[LJMD_MAX_TYPES];
} ljmd_params;

/* ---- neighbor list storage formats (ljmd_nlist.format, set by the build) ----
 * LJMD_FMT_GLOBAL: row i belongs to atom i; entry k of row i is the uint32 at
 *   ((i / 64) * cap + k) * 64 + (i % 64) of neigh: rows are interleaved
 *   across consecutive atoms (Sec. 4.1: the GPU layout interleaves the lists
 *   of consecutive atoms) in blocks of one 64-lane wavefront.  Bits 0..25
 *   hold the neighbor's atom index j; bits 26+2d..27+2d the image code of
 *   dimension d (0: none, 1: d_ij -= len, 2: d_ij += len, d_ij = x_i - x_j).
 * LJMD_FMT_TILED: rows follow the cell order of the build (row s belongs to
 *   atom perm[s], perm kept in aux) and entries are 16-bit slots into the
 *   stencil of the row's tile (a block of tile[0] x tile[1] x tile[2] cells
 *   handled by one workgroup; the stencil is the block one cell wider on
 *   every side), packed four to a 64-bit word; word w of row s is the uint64
 *   at ((s / 64) * capw + w) * 64 + (s % 64), capw = 2 * ceil(cap / 8); a
 *   row of nn entries is padded to a multiple of 8 entries with the slot
 *   number one past the tile's last staged atom.  The force and adjoint
 *   kernels stage a tile's stencil atoms in LDS and read partners from there.
 *   Chosen whenever every dimension has at least 3 cells (unless
 *   LJMD_NL_GLOBAL is set); ljmd_nl_export converts it to the global form.
 * In both formats the order of entries inside a row is unspecified. */
#define LJMD_FMT_GLOBAL 0
#define LJMD_FMT_TILED 1
#define LJMD_NL_GLOBAL 1 /* ljmd_nlist.flags (input): always build the global
                            format */
#define LJMD_NL_SORTED 2 /* ljmd_nlist.flags (output): set by a build that
                            reordered the atoms into cell order (md_step with
                            LJMD_SORT), so that row s belongs to atom s;
                            cleared by every other build */

/* Verlet neighbor list (host struct holding device pointers).
 *  numneigh[n]   int32, entries used in each row (<= cap).
 *  neigh[]       uint32, ljmd_nlist_entries(n, cap) elements, holding the
 *                rows in the format recorded in `format`.
 *  status[4]     int32 status words (LJMD_ST_*).
 *  xref[n][3]    float64 positions at the last build, used by md_step to
 *                detect an unsafe rebuild interval; may be NULL.
 *  aux           ljmd_nlist_aux_bytes(n, box, params) bytes of device memory
 *                that the list keeps its cell order in (aux_bytes: its size).
 * n, mode, cap, flags and the pointers are inputs; format, tile and ncell
 * are written by the build (tile: cells per workgroup along x, y, z) and
 * checked by the readers of the list (a list is only valid for the box and
 * cutoffs it was built with).  All arrays are caller-owned device memory. */
typedef struct {
    int64_t n;
    int32_t mode;
    int32_t cap;
    int32_t *numneigh;
    uint32_t *neigh;
    int32_t *status;
    double *xref;
    void *aux;
    size_t aux_bytes;
    int32_t flags;
    int32_t format;
    int32_t tile[3];
    int32_t ncell[3];
} ljmd_nlist;

/* Number of uint32 elements of ljmd_nlist.neigh for n atoms and capacity cap
 * (n rounded up to a multiple of 64, times cap rounded up to a multiple of
 * 16); 0 for n < 0 or cap < 1. */
int64_t ljmd_nlist_entries(int64_t n, int32_t cap);

/* Bytes of ljmd_nlist.aux for this system (0 if the arguments are invalid). */
size_t ljmd_nlist_aux_bytes(int64_t n, const ljmd_box *box, const ljmd_params *p);

/* Write the list in the global format with rows by atom index: out (device
 * uint32[ljmd_nlist_entries(n, cap)]) and counts (device int32[n]).  Entry
 * order within a row is unspecified.  Async on stream. */
int ljmd_nl_export(const ljmd_nlist *nl, uint32_t *out, int32_t *counts, void *stream);

/* Write the list as plain atom indices, one row per atom, entry k of atom i's
 * row at out[k * n + i] (out: device int32[cap * n], k-major, the layout of
 * the interleaved index list of Sec. 4.1 without the per-wave blocking or
 * image codes), counts[i] entries in row i (device int32[n]); entries beyond
 * counts[i] are left as they were.  Entry order within a row is unspecified.
 * Half lists hold each pair once, in the row the build chose (see
 * ljmd_nl_build).  Async on stream.  As for ljmd_nl_export, a tiled batch
 * list is refused (LJMD_EINVAL): it can be read only with its batch. */
int ljmd_nl_export_indices(const ljmd_nlist *nl, int32_t *out, int32_t *counts, void *stream);

/* Bytes of device scratch every compute entry point needs for this system.
 * Returns 0 when the arguments are invalid (see ljmd_nl_build). */
size_t ljmd_workspace_bytes(int64_t n, const ljmd_box *box,
                            const ljmd_params *p, uint32_t flags);

/* Build the neighbor list of x (Sec. 4; full/half per Sec. 4.1).
 * x is wrapped into the box IN PLACE first (x < 0 -> x + len, x >= len ->
 * x - len, len -> 0), then atoms are binned into cells of side at least
 * max(rc_ij + skin) by a stable counting sort, and each atom's 27-cell
 * stencil (de-duplicated when a dimension has fewer than 3 cells) is
 * searched for partners with r < rc_ij + skin, using FP64 distances
 * d = x_i - x_j, minimum image d > len/2 -> d - len, d < -len/2 -> d + len,
 * r^2 = fma(dz,dz, fma(dy,dy, dx*dx)).  Rows longer than nl->cap are cut
 * at cap; the status words record the overflow and the count needed.
 * nl->status is reset by this call.  If nl->xref is set it receives the
 * wrapped positions.  ws: device scratch of ljmd_workspace_bytes(). */
int ljmd_nl_build(double *x, const int32_t *type, int64_t n,
                  const ljmd_box *box, const ljmd_params *p, ljmd_nlist *nl,
                  void *ws, size_t ws_bytes, void *stream);

/* Forces, and optionally energy and virial, over a list built for these
 * atoms (Sec. 4, Eq. (1)).  f[n][3] is overwritten with the force on each
 * atom.  With LJMD_EV, ev (device float64[7], or NULL) receives E, Wxx,
 * Wyy, Wzz, Wxy, Wxz, Wyz where W_ab = sum over pairs of d_a (f_ij)_b.
 * A full list is evaluated by gather (one atom per lane, no atomics); a
 * half list by scatter (FP64 atomic adds on f).  The reductions of E and W
 * are in a fixed order, so the gather path is bitwise reproducible. */
int ljmd_lj_forces(const double *x, const int32_t *type, int64_t n,
                   const ljmd_box *box, const ljmd_params *p,
                   const ljmd_nlist *nl, uint32_t flags, double *f,
                   double *ev, void *ws, size_t ws_bytes, void *stream);

/* Adjoint of the force map at fixed cutoffs: given gF = dL/dF [n][3], write
 * gx = dL/dx [n][3] (the pair Hessian-vector product, -H gF), and geps,
 * gsig (device float64[ntypes*ntypes], row-major, may each be NULL) =
 * dL/deps, dL/dsigma.  For unlike types the parameter gradient is split
 * evenly between [a][b] and [b][a], so the gradient of a shared parameter
 * is the sum of both entries.  Needs a FULL list; FP64 only
 * (LJMD_ENOTSUP otherwise). */
int ljmd_lj_backward(const double *x, const int32_t *type, int64_t n,
                     const ljmd_box *box, const ljmd_params *p,
                     const ljmd_nlist *nl, const double *gF, uint32_t flags,
                     double *gx, double *geps, double *gsig, void *ws,
                     size_t ws_bytes, void *stream);

/* Force-matching gradient in one call (the workload statement's training
 * step): the forces F of the current parameters (LJMD_PREC_MIXED: FP32 pair
 * terms as in ljmd_lj_forces; FP64 otherwise), the loss gradient
 * g_i = w (F_i - f_target_i), and its adjoint as ljmd_lj_backward (FP64) to
 * gx [n][3] and the T x T tables geps, gsig (may be NULL).  weight: NULL for
 * w = 2 / n, the gradient of L = (1/n) sum_i |F_i - f_target_i|^2 (mean over
 * atoms of the squared force error), else a device pointer to one double w.
 * f (may be NULL) receives F.  With a tiled list the force kernel writes g
 * as each atom's force is complete (no separate pass); g lives in the
 * workspace (ljmd_workspace_bytes).  Results are bit-identical to
 * ljmd_lj_forces, g formed as (F - f_target) * w, then ljmd_lj_backward.
 * Full lists only (LJMD_ENOTSUP otherwise). */
int ljmd_fm_grad(const double *x, const int32_t *type, int64_t n, const ljmd_box *box,
                 const ljmd_params *p, const ljmd_nlist *nl, const double *f_target,
                 const double *weight, uint32_t flags, double *f, double *gx, double *geps,
                 double *gsig, void *ws, size_t ws_bytes, void *stream);

/* ljmd_lj_backward without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving or training
 * loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * kernels as ljmd_lj_backward (bit-identical outputs); the adjoint's
 * per-workgroup partial sums go to a static device array of the library
 * instead of ws: LJMD_NOALLOC_MAX_BLOCKS rows of 32 doubles (4 MiB), on
 * every device the library runs on, held until the process ends.  A call
 * needs one row per tile of a tiled list and one per 256 atoms of a global
 * one; beyond LJMD_NOALLOC_MAX_BLOCKS it returns LJMD_ESCRATCH before any
 * HIP call.  The library allocates nothing here (the first call on a device
 * looks up the array's device address).  All calls on one device share the
 * array: calls that overlap in time on one device (different streams, or
 * threads) race and must be serialized by the caller. */
#define LJMD_NOALLOC_MAX_BLOCKS 16384
int ljmd_lj_backward_noalloc(const double *x, const int32_t *type, int64_t n,
                             const ljmd_box *box, const ljmd_params *p,
                             const ljmd_nlist *nl, const double *gF, uint32_t flags,
                             double *gx, double *geps, double *gsig, void *stream);

/* Velocity Verlet, nsteps steps with global step numbers g = step0+1 ...
 * step0+nsteps, mutating x, v, f and nl in place (and, with LJMD_SORT, the
 * order of the atoms: type and id, if given, are permuted with x and v;
 * id[n] is an optional int32 array that lets the caller follow atoms):
 *   v += (dt/2m) f;  x += dt v;
 *   if g % rebuild_every == 0: wrap x and rebuild nl (as ljmd_nl_build);
 *   f = forces(x);  v += (dt/2m) f.
 * Without LJMD_SETUP, nl and f must be current for x on entry; with it the
 * list is built and f computed first.  Thermo rows [g, E, KE, Wxx, Wyy,
 * Wzz, Wxy, Wxz, Wyz] (float64, 9 per row) are written to the device array
 * thermo for every g with g % thermo_every == 0 (g = step0 only with
 * LJMD_SETUP), in step order; thermo_every = 0 disables them.  The status
 * words are reset on entry and accumulate over the call.  With LJMD_SORT the
 * atoms are reordered at every build (set-up included) so that atoms of one
 * cell are contiguous, which makes the neighbor gathers of the force kernel
 * local in memory; f is recomputed right after each build.  With
 * LJMD_SYNC_CHECK the call synchronizes after each rebuild and returns
 * LJMD_ENEIGH_OVERFLOW at the first overflowing rebuild (x and v are then
 * advanced to that step; f and the rest of the step are not).  With a full
 * list in the tiled format the force kernel applies the kicks and the drift
 * itself as each atom's force is done (the same operations as the separate
 * kernels, in the same order), drifting into a workspace copy of x that
 * alternates with x; the final positions are copied back to x before the
 * call returns.  LJMD_SEPARATE_KICK turns this off. */
int ljmd_md_step(double *x, double *v, double *f, int32_t *type, int32_t *id,
                 int64_t n, const ljmd_box *box, const ljmd_params *p,
                 ljmd_nlist *nl, double dt, int64_t step0, int64_t nsteps,
                 int32_t rebuild_every, int32_t thermo_every, uint32_t flags,
                 double *thermo, void *ws, size_t ws_bytes, void *stream);

/* ---- batches of independent systems ----
 * A batch is nrep independent periodic systems that share the force-field
 * parameters (the workload statement's many uneven replicas): system r owns
 * atoms offsets[r] .. offsets[r+1]-1 of the batch-wide arrays x, v, f, type,
 * id and has its own box boxes[r] (each length at least 2 max(rc + skin) and
 * below 1e9, as for one system).  The caller passes host copies of offsets
 * and boxes (used to size buffers and grids) and identical device copies
 * (read by the kernels); keeping them equal is the caller's duty.  Every
 * call covers all systems with one launch per kernel.  Batch lists are full
 * lists (LJMD_FULL), tiled or in the global format (see
 * ljmd_batch_nl_build); the build sets LJMD_NL_BATCH in flags, the total
 * cell count in ncell[0] and nrep in ncell[1], and the readers check them.
 * Atom sorting (LJMD_SORT) reorders atoms inside each system.  Energies,
 * virials and thermo rows are per system.  Errors as for one system; a half
 * list gives LJMD_ENOTSUP. */
typedef struct {
    int32_t nrep;              /* systems, >= 1 */
    int32_t tile_atoms;        /* home atoms a tile of a tiled batch list (and a
                                  strip of the global build) is cut for: 0 for
                                  the default 300, else 32 .. 4096; a list is
                                  read only with the value it was built with
                                  (kept in its tile[0]) */
    const int64_t *offsets;    /* host int64[nrep + 1]; offsets[0] = 0, non-decreasing */
    const double *boxes;       /* host double[nrep][3] */
    const int64_t *d_offsets;  /* device copy of offsets */
    const double *d_boxes;     /* device copy of boxes */
} ljmd_batch;

#define LJMD_NL_BATCH 4 /* ljmd_nlist.flags (output): built by ljmd_batch_nl_build */

/* Force-kernel variant of the batch path: lanes sharing one atom's list
 * (1, 2 or 4; or 0, which on a tiled list chooses per tile the most lanes
 * that cover the tile's atoms in one pass and on a global list acts as 1),
 * workgroup size (128 or 256), and, when persistent > 0, a grid of
 * persistent x (compute units) workgroups striding over the atoms, or over
 * the tiles of a tiled list (0: one workgroup per group of atoms, or per
 * tile).  On a tiled batch list (512-lane workgroups) block does not
 * apply. */
typedef struct {
    int32_t lanes_per_atom;
    int32_t block;
    int32_t persistent;
    int32_t tile_atoms; /* the batch tiling the variant was chosen for (output of
                           ljmd_batch_autotune; ignored on input) */
} ljmd_batch_tuning;

#define LJMD_TUNE_TILES (1u << 6) /* ljmd_batch_autotune: also search the tile
                                     target (rebuilds the list) */
#define LJMD_TUNE_MD (1u << 7)    /* with LJMD_TUNE_TILES: weigh the tiling for
                                     the MD step (force + build / 20), not for
                                     the force-matching gradient */

/* Bytes of device scratch / list aux for a batch (0 if the arguments are
 * invalid). */
size_t ljmd_batch_workspace_bytes(const ljmd_batch *b, const ljmd_params *p, uint32_t flags);
size_t ljmd_batch_aux_bytes(const ljmd_batch *b, const ljmd_params *p);

/* Wrap every system's atoms into its box and build the batch list (full).
 * nl->n is the batch's total atom count.  The list is in the tiled format
 * (each system cut into tiles along x of about 200 atoms, the systems' tiles
 * numbered one after the other; one workgroup per tile in every reader) unless
 * nl->flags has LJMD_NL_GLOBAL, which selects the global format with
 * batch-wide atom indices. */
int ljmd_batch_nl_build(double *x, const int32_t *type, const ljmd_batch *b,
                        const ljmd_params *p, ljmd_nlist *nl, void *ws, size_t ws_bytes,
                        void *stream);

/* Forces of all systems (FP64, or LJMD_PREC_MIXED); with LJMD_EV and ev
 * non-NULL, ev[r][7] = E, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz of system r.  Uses the
 * variant chosen by ljmd_batch_autotune / ljmd_batch_set_tuning for this
 * batch size, else lanes_per_atom 0 on a tiled list and 1, block 256,
 * persistent 0 on a global one. */
int ljmd_batch_lj_forces(const double *x, const int32_t *type, const ljmd_batch *b,
                         const ljmd_params *p, const ljmd_nlist *nl, uint32_t flags, double *f,
                         double *ev, void *ws, size_t ws_bytes, void *stream);

/* Write a batch list (either format) in the global format with batch-wide
 * atom indices, as ljmd_nl_export does for one system (a tiled batch list
 * can only be read with its batch).  ws: ljmd_batch_workspace_bytes bytes. */
int ljmd_batch_nl_export(const ljmd_nlist *nl, const ljmd_batch *b, const ljmd_params *p,
                         uint32_t *out, int32_t *counts, void *ws, size_t ws_bytes,
                         void *stream);

/* Adjoint of the batch forces (FP64 only): gx as ljmd_lj_backward per
 * system; geps / gsig (T x T, may be NULL) summed over all systems. */
int ljmd_batch_lj_backward(const double *x, const int32_t *type, const ljmd_batch *b,
                           const ljmd_params *p, const ljmd_nlist *nl, const double *gF,
                           uint32_t flags, double *gx, double *geps, double *gsig, void *ws,
                           size_t ws_bytes, void *stream);

/* Force-matching gradient of all systems in one call, as ljmd_fm_grad per
 * system: the loss is sum_r (w_r / 2) sum_{i in r} |F_i - f_target_i|^2
 * with weight[r] (device array of nrep doubles) or, with weight NULL,
 * w_r = 2 / N_r (each system's mean squared force error, summed over the
 * systems); geps / gsig are summed over the systems.  LJMD_PREC_MIXED
 * applies to the forward forces only. */
int ljmd_batch_fm_grad(const double *x, const int32_t *type, const ljmd_batch *b,
                       const ljmd_params *p, const ljmd_nlist *nl, const double *f_target,
                       const double *weight, uint32_t flags, double *f, double *gx,
                       double *geps, double *gsig, void *ws, size_t ws_bytes, void *stream);

/* Velocity Verlet for all systems, as ljmd_md_step; thermo rows are
 * thermo[row][r][9] (row as for one system, r the system).  With a tiled
 * batch list the gather applies the velocity-Verlet updates as for one
 * system (the workspace holds the second position buffer; the final
 * positions are back in x on return); on thermo steps it applies only the
 * second half kick, so the rows see full-step velocities.  LJMD_SEPARATE_KICK
 * turns this off (results are bit-identical).  No host synchronization
 * unless LJMD_SYNC_CHECK, so the call can be captured in a HIP graph. */
int ljmd_batch_md_step(double *x, double *v, double *f, int32_t *type, int32_t *id,
                       const ljmd_batch *b, const ljmd_params *p, ljmd_nlist *nl, double dt,
                       int64_t step0, int64_t nsteps, int32_t rebuild_every,
                       int32_t thermo_every, uint32_t flags, double *thermo, void *ws,
                       size_t ws_bytes, void *stream);

/* Time every force variant on this batch and list (6 runs each, the first
 * discarded and the fastest of the others kept; f is overwritten), keep the
 * fastest variant for later batch calls of
 * the same class -- atom count (power-of-two bucket), expected neighbors per
 * atom ((4 pi / 3) max(rc + skin)^3 times the batch density, bucket of 8),
 * tile target, precision (LJMD_PREC_MIXED in flags) and list format -- and
 * return it in *best (may be NULL).  With LJMD_TUNE_TILES and a tiled list
 * the tile target is searched too (150, 200, 300, 450 and 600 home atoms per
 * tile, those whose workspace and list aux fit ws_bytes and nl->aux_bytes):
 * for each the list is rebuilt (x is wrapped in place, a no-op for wrapped
 * positions) and the build, the force variants and the FP64 adjoint are
 * timed; the cost minimized is force + adjoint + build / 20 (a rebuild every
 * 20 steps), or force + build / 20 with LJMD_TUNE_MD.  nl is then left built for the chosen target
 * (best->tile_atoms), sorted-marked if it was and its atoms kept their
 * places; later calls must pass a batch with that tile_atoms.  Synchronizes
 * `stream`.  Process-wide table. */
int ljmd_batch_autotune(double *x, const int32_t *type, const ljmd_batch *b,
                        const ljmd_params *p, ljmd_nlist *nl, uint32_t flags, double *f,
                        void *ws, size_t ws_bytes, void *stream, ljmd_batch_tuning *best);

/* Set (t non-NULL) or clear (t NULL) the variant used for this batch size and
 * precision.  LJMD_EINVAL for a variant outside the list above. */
int ljmd_batch_set_tuning(const ljmd_batch *b, const ljmd_params *p, uint32_t flags,
                          const ljmd_batch_tuning *t);

/* Lanes that share one atom's row in the full-list force gather and in the
 * adjoint over a tiled list: 1, 2, 4 or 8, or 0 (the default) to choose them
 * automatically: the adjoint per tile (the most lanes that cover the tile's
 * home atoms in one pass of a 512-lane workgroup), the gather of one system
 * the same way for tiles of fewer than about 200 atoms (which small systems
 * get so that there are enough workgroups to fill the GPU) and otherwise
 * from the list's tile size (2 for tiles of about half a workgroup, else 1);
 * the batch gather follows the batch tuning instead of this setting.  Lane
 * k of an atom takes the list words
 * k, k + lanes, ... and the partial results are summed over the lanes in a
 * fixed order, so results are reproducible for a given setting and differ
 * between settings only by summation order.  Process-wide; takes effect for
 * calls made after it returns.  LJMD_EINVAL for any other value. */
int ljmd_set_gather_lanes(int lanes);

/* The current setting of ljmd_set_gather_lanes (0: automatic). */
int ljmd_get_gather_lanes(void);

/* Lanes per atom the force gather uses on this built list with the current
 * setting (1 for the global format, 0 when they are chosen per tile), or a
 * negative LJMD_E* code if the list was not built for this box and these
 * cutoffs.  Host only. */
int ljmd_nl_gather_lanes(const ljmd_nlist *nl, const ljmd_box *box, const ljmd_params *p);

/* Copy the status words of nl to host out[4]; synchronizes `stream`. */
int ljmd_get_status(const ljmd_nlist *nl, int32_t *out, void *stream);

/* Static description of a return code (never NULL). */
const char *ljmd_strerror(int code);

/* Text of the last HIP error seen by this library in this thread. */
const char *ljmd_last_hip_error(void);

/* ---- measurement hooks ----
 * With profiling on, every entry point brackets each of its phases with a
 * pair of HIP events recorded on its stream; ljmd_profile_read waits for the
 * recorded events, adds up the elapsed GPU time per phase, and clears the
 * record.  Phases: LJMD_PHASE_FORCE (the force kernel, plus the zeroing of f
 * for a half list), LJMD_PHASE_BUILD (binning and neighbor build),
 * LJMD_PHASE_INTEGRATE (velocity-Verlet kernels), LJMD_PHASE_OTHER
 * (reductions, status and thermo rows).  Process-wide; not for concurrent
 * use from several threads. */
#define LJMD_PHASE_FORCE 0
#define LJMD_PHASE_BUILD 1
#define LJMD_PHASE_INTEGRATE 2
#define LJMD_PHASE_OTHER 3
#define LJMD_PHASES 4

/* Turn profiling on (1) or off (0); returns LJMD_OK. */
int ljmd_profile_enable(int on);

/* Host out: ms[LJMD_PHASES] total GPU milliseconds and launches[LJMD_PHASES]
 * bracketed phase instances since the last read.  Synchronizes with the
 * recorded events.  LJMD_EHIP on a HIP failure. */
int ljmd_profile_read(double *ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif
