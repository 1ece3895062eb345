// Internal definitions shared by the HIP kernels and the C-ABI layer of
// libljmd.  Nothing here is part of the public interface (include/ljmd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ljmd {

constexpr int kMaxTypes = 4;
constexpr int kTab = kMaxTypes * kMaxTypes;
constexpr uint32_t kIndexMask = (1u << 26) - 1u;  // bits 0..25: atom index
constexpr int kCodeShift = 26;                    // bits 26..31: image code
constexpr int kWave = 64;                         // CDNA wavefront width
constexpr int kXcds = 8;                          // MI355X: 8 XCDs, round-robin dispatch

// Periodic orthorhombic box: lengths and half lengths.
struct Box {
    double L[3];
    double hL[3];
};

// Uniform cell grid over the box.
struct Grid {
    int nc[3];        // cells per dimension (>= 1)
    double cinv[3];   // nc / L
    int64_t ncell;
};

// Per-type-pair constants, indexed ti * ntypes + tj, passed by value.
//   rnb2 = (rc + skin)^2, rc2 = rc^2,
//   lj1 = 48 eps sigma^12, lj2 = 24 eps sigma^6   (force),
//   lj3 =  4 eps sigma^12, lj4 =  4 eps sigma^6   (energy).
struct PairTab {
    int ntypes;
    int pad;
    double rnb2[kTab];
    double rc2[kTab];
    double lj1[kTab];
    double lj2[kTab];
    double lj3[kTab];
    double lj4[kTab];
    double eps[kTab];
    double sig[kTab];
    float lj1f[kTab];
    float lj2f[kTab];
    float lj3f[kTab];
    float lj4f[kTab];
};

// Offsets (bytes) of the scratch regions inside the caller's workspace.
struct Workspace {
    size_t scan_bsum;    // int32[scan blocks + 1]
    size_t atom_cell;    // int32[n]
    size_t atom_slot;    // int32[n]
    size_t tmp;          // int32[n]
    size_t pos;          // double4[n]: cell-sorted wrapped positions, w = type
    size_t part_a;       // double[blocks * kPartVals]: per-block partial sums
    size_t part_b;       // double[blocks]: per-block kinetic partial sums
    size_t sort_v;       // double[3n]: velocities in cell order (atom sorting)
    size_t sort_i;       // int32[2n]: types and ids in cell order (atom sorting)
    size_t xalt;         // double[3n]: second position buffer of the fused step
    size_t total;
    int64_t part_a_blocks;
    int64_t part_b_blocks;
};

// Offsets (bytes) inside a neighbor list's aux buffer (state that belongs to
// the list: the cell order it was built in).
struct Aux {
    size_t perm;        // int32[n]: cell-sorted position -> atom index
    size_t cell_start;  // int32[ncell + 1]: cell-sorted start of every cell
    size_t total;
};

// One system of a batch of independent periodic systems (a device table
// filled by the batch plan kernel from the caller's offsets and boxes).
struct RepInfo {
    Box box;
    Grid g;
    int64_t atom_base, natoms;
    int64_t cell_base;  // first cell of this system in the batch-wide cell order
    int64_t item_base;  // first neighbor-build work item of this system
    int64_t tile_base;  // first tile of this system in a tiled list
    int32_t strip;      // build strip length along x (cells)
    int32_t nstripx;    // strips per grid row
    int32_t small;      // some dimension has fewer than 3 cells
    int32_t ey;         // cells along y of a tiled list's tiles
};

constexpr int kScanItems = 1024;  // elements per scan block (256 threads x 4)
constexpr int kPartVals = 32;     // doubles reserved per block in part_a

// Block index remap so that each XCD (which owns its own L2) receives one
// contiguous range of logical blocks.  Hardware hands block b to XCD b % 8.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    const int64_t q = nb / kXcds, r = nb % kXcds;
    const int64_t x = b % kXcds, l = b / kXcds;
    return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// Entry k of row i in the wave-interleaved neighbor layout.
__device__ __forceinline__ int64_t nl_slot(int64_t i, int64_t k, int cap) {
    return ((i >> 6) * (int64_t)cap + k) * kWave + (i & 63);
}

// Wave64 sum / max reductions (all lanes receive the result).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// Velocity-Verlet update applied by the full-list gather to each atom as
// soon as its force is complete (mode 0: none).  mode 1: v += h f (the
// second half kick of a step); mode 2: that, then the next step's half kick
// v += h f and drift xnext = x + dt v, written to a separate buffer because
// other workgroups are still reading x.  h = dt / (2 m) per type.  The
// kinetic energy after the second half kick goes into slot 7 of the
// energy/virial partials, and a non-finite velocity sets status[3].
struct Kick {
    double *v;
    double *xnext;
    int32_t *status;
    double h[kMaxTypes];
    double mass[kMaxTypes];
    double dt;
    int mode;
};

// Force-matching output of the full-list gather (g == nullptr: none).  As
// soon as an atom's force F_i is complete the gather writes the gradient of
// the loss sum_r (w_r / 2) sum_{i in r} |F_i - Ft_i|^2 with respect to it,
// g_i = w_r (F_i - Ft_i), where w_r = wsys[r] (one value per system, wsys[0]
// for a single system) or, with wsys null, 2 / (atoms of the system): the
// mean-over-atoms loss.  The forces themselves are then written only when
// the kernel's f is non-null.
struct FmOut {
    const double *ft;
    const double *wsys;
    double *g;
};

// ---- launchers (defined in the .hip files) ----
struct TileArgs;
hipError_t launch_zero_i32(int32_t *p, int64_t len, hipStream_t s);
hipError_t launch_zero_f64(double *p, int64_t len, hipStream_t s);
hipError_t launch_set_i32(int32_t *p, int64_t len, int32_t value, hipStream_t s);
hipError_t launch_bin(double *x, const int32_t *type, int64_t n, const Box &box,
                      const Grid &g, double *xref, char *ws, const Workspace &w,
                      int32_t *cell_start, int32_t *perm, hipStream_t s,
                      const RepInfo *reps = nullptr, const int32_t *rid = nullptr,
                      int64_t ncell_total = 0, double disp_lim2 = 0.0,
                      int32_t *disp_status = nullptr, bool sorting = false);
hipError_t launch_sort(int64_t n, double *x, double *v, int32_t *type, int32_t *id, double *xref,
                       int32_t *perm, char *ws, const Workspace &w, hipStream_t s);
int64_t tile_blocks(const TileArgs &t);
hipError_t launch_nl_build(int64_t n, const TileArgs &t, const PairTab &tab, int half, int tiled,
                           const char *ws, const Workspace &w, void *neigh, int32_t *numneigh,
                           int cap, int32_t *status, hipStream_t s);
hipError_t launch_nl_export(int64_t n, const TileArgs &t, int tiled, const void *neigh,
                            const int32_t *numneigh, int cap, uint32_t *out, int32_t *counts,
                            hipStream_t s, int kmajor = 0);
hipError_t launch_forces(const double *x, const int32_t *type, int64_t n, const Box &box,
                         const PairTab &tab, const int32_t *numneigh, const uint32_t *neigh,
                         int cap, int half, int mixed, int ev, double *f, double *partials,
                         int64_t *nblocks_out, hipStream_t s);
hipError_t launch_forces_tiled(const TileArgs &t, const double *x, const int32_t *type,
                               int64_t n, const PairTab &tab, const int32_t *numneigh,
                               const void *neigh, int cap, int sorted, int half, int mixed, int ev,
                               int lpa, double *f, double *partials, int64_t *nblocks_out,
                               hipStream_t s, const Kick *kick = nullptr,
                               double *ev_atom = nullptr, int persistent = 0,
                               const FmOut *fm = nullptr);
hipError_t launch_reduce_partials(const double *partials, int64_t nblocks, int nvals,
                                  double *out, hipStream_t s);
hipError_t launch_fm_grad(const double *f, const FmOut &fm, int64_t n, const RepInfo *reps,
                          const int32_t *rid, hipStream_t s);
hipError_t launch_backward(const double *x, const int32_t *type, int64_t n, const Box &box,
                           const PairTab &tab, const int32_t *numneigh, const uint32_t *neigh,
                           int cap, const double *gF, double *gx, double *partials,
                           int64_t *nblocks_out, hipStream_t s);
hipError_t launch_backward_tiled(const TileArgs &t, const double *x, const int32_t *type,
                                 int64_t n, const PairTab &tab, const int32_t *numneigh,
                                 const void *neigh, int cap, int sorted, int lpa,
                                 const double *gF, double *gx, double *partials,
                                 int64_t *nblocks_out, hipStream_t s);
hipError_t launch_param_grads(const double *partials, int64_t nblocks, int ntypes,
                              double *geps, double *gsig, hipStream_t s);
// v += h f, then x + dt v into xout (nullptr: into x).
hipError_t launch_kick_drift(double *x, double *v, const double *f, const int32_t *type,
                             int64_t n, const double *dtf, int ntypes, double dt,
                             hipStream_t s, double *xout = nullptr);
hipError_t launch_kick(double *x, double *v, const double *f, const int32_t *type, int64_t n,
                       const double *dtf, const double *mass, int ntypes, double dt,
                       int drift_after, int ke, double *ke_partials, int64_t *nblocks_out,
                       int32_t *status, hipStream_t s);
hipError_t launch_thermo_row(const double *ev_partials, int64_t ev_blocks,
                             const double *ke_partials, int64_t ke_blocks, int64_t step,
                             double *row, hipStream_t s);
// ---- batches of independent systems ----
struct BatchView {
    int32_t nrep;
    const int64_t *offsets;  // device int64[nrep + 1]
    const RepInfo *reps;     // device RepInfo[nrep]
    const int32_t *rid;      // device int32[n]: system of each atom
};
hipError_t launch_batch_plan(int32_t nrep, const int64_t *offsets, const double *boxes,
                             double max_rnb, int tile_atoms, RepInfo *reps, int32_t *rid, int64_t n,
                             int32_t *tile_rep, int64_t ntiles, hipStream_t s);
hipError_t launch_nl_build_batch(int64_t n, const BatchView &b, int64_t nitems,
                                 const int32_t *cell_start, const int32_t *perm,
                                 const PairTab &tab, int half, const char *ws,
                                 const Workspace &w, uint32_t *neigh, int32_t *numneigh, int cap,
                                 int32_t *status, hipStream_t s);
hipError_t launch_forces_batch(const double *x, const int32_t *type, int64_t n,
                               const BatchView &b, const PairTab &tab, const int32_t *numneigh,
                               const uint32_t *neigh, int cap, int mixed, double *f,
                               double *ev_atom, int lanes_per_atom, int block, int persistent,
                               hipStream_t s);
hipError_t launch_backward_batch(const double *x, const int32_t *type, int64_t n,
                                 const BatchView &b, const PairTab &tab, const int32_t *numneigh,
                                 const uint32_t *neigh, int cap, const double *gF, double *gx,
                                 double *partials, int64_t *nblocks_out, hipStream_t s);
hipError_t launch_batch_thermo(const BatchView &b, const double *v, const int32_t *type,
                               const double *mass, int ntypes, const double *ev_atom, int64_t n,
                               int64_t step, double *rows, double *ev_out, hipStream_t s);
hipError_t launch_perm_identity(const int32_t *perm, int64_t n, int32_t *flag, hipStream_t s);

}  // namespace ljmd
