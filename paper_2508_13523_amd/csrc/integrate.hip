// Velocity-Verlet kernels, kinetic-energy partial sums, thermo rows and the
// rebuild-safety check.
//
// The paper only says that MD integrates Newton's second law (Sec. 1); the
// step used here is velocity Verlet with half kicks v += (dt/2m) f around a
// drift x += dt v, each update a single fma.  The second half kick of step s
// and the first half kick and drift of step s+1 use the same forces, so they
// run as one kernel (two separate fmas, bit-identical to running them apart).
#include "common.hpp"

namespace ljmd {

namespace {

constexpr int kThreads = 256;

struct Dtf {
    double h[kMaxTypes];     // dt / (2 m_t)
    double mass[kMaxTypes];
};

// a[t] for a per-lane t, with uniform loads and selects only (no indexed
// access into the kernel-argument struct).
__device__ __forceinline__ double sel4(const double (&a)[kMaxTypes], int t) {
    double r = a[0];
    r = t == 1 ? a[1] : r;
    r = t == 2 ? a[2] : r;
    r = t == 3 ? a[3] : r;
    return r;
}

template <int T>
// (xout may be x: each element is read before it is written, by the same
// thread)
__global__ __launch_bounds__(kThreads) void k_kick_drift(const double *x, double *xout,
                                                         double *__restrict__ v,
                                                         const double *__restrict__ f,
                                                         const int32_t *__restrict__ type,
                                                         int64_t n3, Dtf c, double dt) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n3) return;
    const double h = T > 1 ? sel4(c.h, type[e / 3]) : c.h[0];
    const double vn = fma(h, f[e], v[e]);
    v[e] = vn;
    xout[e] = fma(dt, vn, x[e]);
}

// Second half kick (optionally followed by the next step's half kick and
// drift); v after the second half kick is the full-step velocity, whose
// kinetic energy goes into the per-block partials.
template <int T, bool DRIFT, bool KE>
__global__ __launch_bounds__(kThreads) void k_kick(double *__restrict__ x,
                                                   double *__restrict__ v,
                                                   const double *__restrict__ f,
                                                   const int32_t *__restrict__ type, int64_t n3,
                                                   Dtf c, double dt, double *__restrict__ kep,
                                                   int32_t *__restrict__ status) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    double ke = 0.0;
    bool bad = false;
    if (e < n3) {
        const int t = T > 1 ? type[e / 3] : 0;
        const double h = T > 1 ? sel4(c.h, t) : c.h[0];
        const double fe = f[e];
        const double v1 = fma(h, fe, v[e]);
        bad = !isfinite(v1);
        if (KE) ke = 0.5 * (T > 1 ? sel4(c.mass, t) : c.mass[0]) * v1 * v1;
        if (DRIFT) {
            const double v2 = fma(h, fe, v1);
            v[e] = v2;
            x[e] = fma(dt, v2, x[e]);
        } else {
            v[e] = v1;
        }
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&status[3], 1);
    if (KE) {
        __shared__ double s[kThreads / kWave];
        ke = wave_sum(ke);
        if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = ke;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < kThreads / kWave; ++w) t += s[w];
            kep[blockIdx.x] = t;
        }
    }
}

// Row [step, E, KE, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz] from the per-block partials,
// summed in a fixed order.  Without kinetic partials (kep null) the kinetic
// energy is slot 7 of the energy/virial partials (the fused gather step).
__global__ __launch_bounds__(kThreads) void k_thermo_row(const double *__restrict__ evp,
                                                         int64_t evb,
                                                         const double *__restrict__ kep,
                                                         int64_t keb, int64_t step,
                                                         double *__restrict__ row) {
    __shared__ double s[kThreads];
    for (int v = 0; v < 8; ++v) {
        double t = 0.0;
        if (v < 7 || !kep) {
            for (int64_t b = threadIdx.x; b < evb; b += kThreads) t += evp[b * kPartVals + v];
        } else {
            for (int64_t b = threadIdx.x; b < keb; b += kThreads) t += kep[b];
        }
        s[threadIdx.x] = t;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (v == 0) row[1] = s[0];
            else if (v == 7) row[2] = s[0];
            else row[2 + v] = s[0];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) row[0] = (double)step;
}

Dtf make_dtf(const double *dtf, const double *mass, int ntypes) {
    Dtf c;
    for (int t = 0; t < kMaxTypes; ++t) {
        c.h[t] = t < ntypes ? dtf[t] : 0.0;
        c.mass[t] = (mass && t < ntypes) ? mass[t] : 0.0;
    }
    return c;
}

template <int T>
hipError_t kick_t(double *x, double *v, const double *f, const int32_t *type, int64_t n3,
                  const Dtf &c, double dt, int drift, int ke, double *kep, int32_t *status,
                  unsigned blocks, hipStream_t s) {
    if (drift) {
        if (ke) k_kick<T, true, true><<<blocks, kThreads, 0, s>>>(x, v, f, type, n3, c, dt, kep, status);
        else k_kick<T, true, false><<<blocks, kThreads, 0, s>>>(x, v, f, type, n3, c, dt, kep, status);
    } else {
        if (ke) k_kick<T, false, true><<<blocks, kThreads, 0, s>>>(x, v, f, type, n3, c, dt, kep, status);
        else k_kick<T, false, false><<<blocks, kThreads, 0, s>>>(x, v, f, type, n3, c, dt, kep, status);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_kick_drift(double *x, double *v, const double *f, const int32_t *type,
                             int64_t n, const double *dtf, int ntypes, double dt, hipStream_t s,
                             double *xout) {
    if (n <= 0) return hipSuccess;
    const Dtf c = make_dtf(dtf, nullptr, ntypes);
    const int64_t n3 = 3 * n;
    const unsigned blocks = (unsigned)((n3 + kThreads - 1) / kThreads);
    double *xo = xout ? xout : x;
    if (ntypes > 1)
        k_kick_drift<2><<<blocks, kThreads, 0, s>>>(x, xo, v, f, type, n3, c, dt);
    else
        k_kick_drift<1><<<blocks, kThreads, 0, s>>>(x, xo, v, f, type, n3, c, dt);
    return hipGetLastError();
}

hipError_t launch_kick(double *x, double *v, const double *f, const int32_t *type, int64_t n,
                       const double *dtf, const double *mass, int ntypes, double dt,
                       int drift_after, int ke, double *ke_partials, int64_t *nblocks_out,
                       int32_t *status, hipStream_t s) {
    const int64_t n3 = 3 * n;
    const int64_t blocks = (n3 + kThreads - 1) / kThreads;
    *nblocks_out = blocks;
    if (n <= 0) return hipSuccess;
    const Dtf c = make_dtf(dtf, mass, ntypes);
    if (ntypes > 1)
        return kick_t<2>(x, v, f, type, n3, c, dt, drift_after, ke, ke_partials, status,
                         (unsigned)blocks, s);
    return kick_t<1>(x, v, f, type, n3, c, dt, drift_after, ke, ke_partials, status,
                     (unsigned)blocks, s);
}

hipError_t launch_thermo_row(const double *ev_partials, int64_t ev_blocks,
                             const double *ke_partials, int64_t ke_blocks, int64_t step,
                             double *row, hipStream_t s) {
    k_thermo_row<<<1, kThreads, 0, s>>>(ev_partials, ev_blocks, ke_partials, ke_blocks, step,
                                        row);
    return hipGetLastError();
}

}  // namespace ljmd
