/*
 * ljref.h -- plain serial FP64 CPU oracle for the Lennard-Jones MD hot path.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  The oracle is the slow, obviously
 * correct definition that the HIP library is checked against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or helper with the HIP library.
 *
 * Source: Johansson, Weinberg, Trott, McCarthy, Moore, "LAMMPS-KOKKOS:
 * Performance Portable Molecular Dynamics Across Exascale Architectures",
 * arXiv:2508.13523.
 *
 * Conventions (all arrays row-major, caller-owned host memory):
 *   x[n][3], v[n][3], f[n][3]   FP64 positions, velocities, forces
 *   type[n]                      int32 in [0, ntypes)
 *   box[3]                       orthorhombic periodic box lengths, origin 0
 *   eps, sigma, rc [ntypes*ntypes]  symmetric per-type-pair tables
 *   ev[7]                        E, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz
 *   Neighbor rows are CSR: counts[n] then idx[] at the caller's offsets.
 *
 * Readings of the paper used here (the paper is silent on these points):
 *   - strict "<" for both the force cutoff and the neighbor cutoff (Eq. (1));
 *   - truncated, unshifted energy, no tail correction (Eq. (1) as written);
 *   - neighbor cutoff per type pair is rc_ij + skin;
 *   - minimum image in branch form: d = xi - xj; d > L/2 -> d - L,
 *     d < -L/2 -> d + L; rsq = fma(dz,dz, fma(dy,dy, dx*dx));
 *   - wrap in branch form: x < 0 -> x + L, x >= L -> x - L, and L -> 0;
 *   - half-list pair (i,j) is stored in row min(i,j);
 *   - virial W_ab = sum over pairs i<j of d_a * (f_ij)_b, d = xi - xj.
 */
#ifndef LJREF_H
#define LJREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

void ref_wrap(int64_t n, double *x, const double *box);

int64_t ref_nl_brute(int64_t n, const double *x, const int32_t *type,
                     const double *box, int32_t ntypes, const double *rc,
                     double skin, int32_t half, int64_t *counts,
                     const int64_t *offsets, int32_t *idx);
int64_t ref_nl_cells(int64_t n, const double *x, const int32_t *type,
                     const double *box, int32_t ntypes, const double *rc,
                     double skin, int32_t half, int64_t *counts,
                     const int64_t *offsets, int32_t *idx);
int64_t ref_nl_rows(int64_t n, const double *x, const int32_t *type,
                    const double *box, int32_t ntypes, const double *rc,
                    double skin, int64_t nrows, const int64_t *rows,
                    int64_t *counts, const int64_t *offsets, int32_t *idx);

void ref_forces_brute(int64_t n, const double *x, const int32_t *type,
                      const double *box, int32_t ntypes, const double *eps,
                      const double *sigma, const double *rc, double *f,
                      double *ev);
void ref_forces_cells(int64_t n, const double *x, const int32_t *type,
                      const double *box, int32_t ntypes, const double *eps,
                      const double *sigma, const double *rc, double *f,
                      double *ev);
void ref_force_rows(int64_t n, const double *x, const int32_t *type,
                    const double *box, int32_t ntypes, const double *eps,
                    const double *sigma, const double *rc, int64_t nrows,
                    const int64_t *rows, double *frows);

void ref_backward_brute(int64_t n, const double *x, const int32_t *type,
                        const double *box, int32_t ntypes, const double *eps,
                        const double *sigma, const double *rc, const double *g,
                        double *gx, double *geps, double *gsig);
void ref_backward_cells(int64_t n, const double *x, const int32_t *type,
                        const double *box, int32_t ntypes, const double *eps,
                        const double *sigma, const double *rc, const double *g,
                        double *gx, double *geps, double *gsig);

double ref_kinetic(int64_t n, const double *v, const int32_t *type,
                   const double *mass);

int64_t ref_md(int64_t n, double *x, double *v, double *f,
               const int32_t *type, const double *box, int32_t ntypes,
               const double *eps, const double *sigma, const double *rc,
               const double *mass, double skin, double dt, int64_t step0,
               int64_t nsteps, int32_t rebuild_every, int32_t thermo_every,
               int32_t setup, double *thermo);

/* ref_md from a fresh set-up (step 0) with the velocities rescaled to the
 * kinetic temperature `temp` after every step (equilibration of inputs). */
int64_t ref_md_rescale(int64_t n, double *x, double *v, double *f,
                       const int32_t *type, const double *box, int32_t ntypes,
                       const double *eps, const double *sigma, const double *rc,
                       const double *mass, double skin, double dt, int64_t nsteps,
                       int32_t rebuild_every, double temp);

#ifdef __cplusplus
}
#endif
#endif
