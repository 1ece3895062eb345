"""numpy front end of the CPU oracle (test infrastructure, not product code).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  It loads ``libljref.so`` (built from
``ljref.c`` by ``oracle/build.py``) and shares nothing with the HIP library.

All arrays are float64 / int32 numpy arrays; parameter tables are
``ntypes x ntypes`` symmetric arrays.  Neighbor lists come back as CSR
``(counts, offsets, idx)`` with every row sorted ascending.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None
_LIB_TIMING = None

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.POINTER(ctypes.c_int64)
_n = ctypes.c_int64


def lib(timing: bool = False):
    """Load (building on first use if needed) the oracle library.  timing=True
    loads the same source built with -O3 -march=native (libljref_timing.so),
    used only to time the oracle; every parity check uses the plain build.
    The timing build is compiled afresh on first use in each process, so that
    -march=native targets the CPU the timing runs on."""
    global _LIB, _LIB_TIMING
    if timing:
        if _LIB_TIMING is None:
            from oracle import build as _b  # noqa: WPS433 (build on demand)
            _LIB_TIMING = _declare(ctypes.CDLL(_b.build_timing()))
        return _LIB_TIMING
    if _LIB is None:
        path = os.path.join(_HERE, "libljref.so")
        src = os.path.join(_HERE, "ljref.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            from oracle import build as _b  # noqa: WPS433 (build on demand)
            _b.build()
        _LIB = _declare(ctypes.CDLL(path))
    return _LIB


def _declare(L):
    """ctypes signatures of the oracle's entry points (ljref.h)."""
    nl = [_n, _d, _i32, _d, ctypes.c_int32, _d, ctypes.c_double, ctypes.c_int32,
          _i64, _i64, _i32]
    L.ref_wrap.argtypes = [_n, _d, _d]
    L.ref_wrap.restype = None
    for name in ("ref_nl_brute", "ref_nl_cells"):
        getattr(L, name).argtypes = nl
        getattr(L, name).restype = ctypes.c_int64
    L.ref_nl_rows.argtypes = [_n, _d, _i32, _d, ctypes.c_int32, _d, ctypes.c_double,
                              _n, _i64, _i64, _i64, _i32]
    L.ref_nl_rows.restype = ctypes.c_int64
    fa = [_n, _d, _i32, _d, ctypes.c_int32, _d, _d, _d, _d, _d]
    for name in ("ref_forces_brute", "ref_forces_cells"):
        getattr(L, name).argtypes = fa
        getattr(L, name).restype = None
    L.ref_force_rows.argtypes = [_n, _d, _i32, _d, ctypes.c_int32, _d, _d, _d, _n, _i64, _d]
    L.ref_force_rows.restype = None
    ba = [_n, _d, _i32, _d, ctypes.c_int32, _d, _d, _d, _d, _d, _d, _d]
    for name in ("ref_backward_brute", "ref_backward_cells"):
        getattr(L, name).argtypes = ba
        getattr(L, name).restype = None
    L.ref_kinetic.argtypes = [_n, _d, _i32, _d]
    L.ref_kinetic.restype = ctypes.c_double
    L.ref_md.argtypes = [_n, _d, _d, _d, _i32, _d, ctypes.c_int32, _d, _d, _d, _d,
                         ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                         ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _d]
    L.ref_md.restype = ctypes.c_int64
    L.ref_md_rescale.argtypes = [_n, _d, _d, _d, _i32, _d, ctypes.c_int32, _d, _d, _d, _d,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                 ctypes.c_int32, ctypes.c_double]
    L.ref_md_rescale.restype = ctypes.c_int64
    return L


def _pd(a):
    return a.ctypes.data_as(_d)


def _pi32(a):
    return a.ctypes.data_as(_i32)


def _pi64(a):
    return a.ctypes.data_as(_i64)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _types(t, n):
    if t is None:
        return np.zeros(n, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    assert t.shape == (n,)
    return t


def _table(a):
    a = np.ascontiguousarray(np.atleast_2d(np.asarray(a, dtype=np.float64)))
    assert a.shape[0] == a.shape[1]
    return a


def wrap(x, box):
    """Positions wrapped into [0, L) (branch form)."""
    x = _f64(x).copy()
    lib().ref_wrap(x.shape[0], _pd(x), _pd(_f64(box)))
    return x


def _nl(fn, x, types, box, rc, skin, half):
    x = _f64(x)
    n = x.shape[0]
    t = _types(types, n)
    rc = _table(rc)
    box = _f64(box)
    counts = np.zeros(n, dtype=np.int64)
    tot = fn(n, _pd(x), _pi32(t), _pd(box), rc.shape[0], _pd(rc), float(skin), int(half),
             _pi64(counts), None, None)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    idx = np.zeros(max(tot, 1), dtype=np.int32)
    fn(n, _pd(x), _pi32(t), _pd(box), rc.shape[0], _pd(rc), float(skin), int(half),
       _pi64(counts), _pi64(offsets), _pi32(idx))
    return counts, offsets, idx[:tot]


def nl_brute(x, types, box, rc, skin, half=False):
    """O(n^2) neighbor list: rows of j with |d_ij| < rc_ij + skin."""
    return _nl(lib().ref_nl_brute, x, types, box, rc, skin, half)


def nl_cells(x, types, box, rc, skin, half=False):
    """Same list via the oracle's own cell grid (O(n))."""
    return _nl(lib().ref_nl_cells, x, types, box, rc, skin, half)


def nl_rows(x, types, box, rc, skin, rows):
    """Full-list rows of the selected atoms, brute force."""
    x = _f64(x)
    n = x.shape[0]
    t = _types(types, n)
    rc = _table(rc)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    counts = np.zeros(rows.shape[0], dtype=np.int64)
    tot = lib().ref_nl_rows(n, _pd(x), _pi32(t), _pd(_f64(box)), rc.shape[0], _pd(rc),
                            float(skin), rows.shape[0], _pi64(rows), _pi64(counts), None, None)
    offsets = np.zeros(rows.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    idx = np.zeros(max(tot, 1), dtype=np.int32)
    lib().ref_nl_rows(n, _pd(x), _pi32(t), _pd(_f64(box)), rc.shape[0], _pd(rc), float(skin),
                      rows.shape[0], _pi64(rows), _pi64(counts), _pi64(offsets), _pi32(idx))
    return counts, offsets, idx[:tot]


def _forces(fn, x, types, box, eps, sigma, rc):
    x = _f64(x)
    n = x.shape[0]
    t = _types(types, n)
    eps, sigma, rc = _table(eps), _table(sigma), _table(rc)
    f = np.zeros((n, 3), dtype=np.float64)
    ev = np.zeros(7, dtype=np.float64)
    fn(n, _pd(x), _pi32(t), _pd(_f64(box)), eps.shape[0], _pd(eps), _pd(sigma), _pd(rc),
       _pd(f), _pd(ev))
    return f, ev


def forces_brute(x, types, box, eps, sigma, rc):
    """Forces [n,3] and ev = (E, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz), all pairs."""
    return _forces(lib().ref_forces_brute, x, types, box, eps, sigma, rc)


def forces_cells(x, types, box, eps, sigma, rc):
    """Same as forces_brute, pairs from the oracle's cell grid."""
    return _forces(lib().ref_forces_cells, x, types, box, eps, sigma, rc)


def force_rows(x, types, box, eps, sigma, rc, rows):
    """Forces on the selected atoms only, brute force over all partners."""
    x = _f64(x)
    n = x.shape[0]
    t = _types(types, n)
    eps, sigma, rc = _table(eps), _table(sigma), _table(rc)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros((rows.shape[0], 3), dtype=np.float64)
    lib().ref_force_rows(n, _pd(x), _pi32(t), _pd(_f64(box)), eps.shape[0], _pd(eps),
                         _pd(sigma), _pd(rc), rows.shape[0], _pi64(rows), _pd(out))
    return out


def _bwd(fn, x, types, box, eps, sigma, rc, g):
    x = _f64(x)
    n = x.shape[0]
    t = _types(types, n)
    eps, sigma, rc = _table(eps), _table(sigma), _table(rc)
    g = _f64(g, (n, 3))
    T = eps.shape[0]
    gx = np.zeros((n, 3))
    geps = np.zeros((T, T))
    gsig = np.zeros((T, T))
    fn(n, _pd(x), _pi32(t), _pd(_f64(box)), T, _pd(eps), _pd(sigma), _pd(rc), _pd(g),
       _pd(gx), _pd(geps), _pd(gsig))
    return gx, geps, gsig


def backward_brute(x, types, box, eps, sigma, rc, g):
    """Adjoint of the force map: (dL/dx, dL/deps, dL/dsigma) given g = dL/dF."""
    return _bwd(lib().ref_backward_brute, x, types, box, eps, sigma, rc, g)


def backward_cells(x, types, box, eps, sigma, rc, g):
    """Same as backward_brute, pairs from the oracle's cell grid."""
    return _bwd(lib().ref_backward_cells, x, types, box, eps, sigma, rc, g)


def kinetic(v, types, mass):
    v = _f64(v)
    n = v.shape[0]
    return lib().ref_kinetic(n, _pd(v), _pi32(_types(types, n)), _pd(_f64(mass)))


def md(x, v, types, box, eps, sigma, rc, mass, dt, nsteps, rebuild_every=20,
       thermo_every=0, step0=0, setup=True, f=None, skin=None, timing=False):
    """Velocity-Verlet run on copies; returns (x, v, f, thermo[rows, 9]).

    skin=None: forces are the exact pair sum every step.  skin >= 0: forces are
    the pair sum over a Verlet list of cutoff rc + skin rebuilt every
    rebuild_every steps (the method as run on the GPU)."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    n = x.shape[0]
    t = _types(types, n)
    eps, sigma, rc = _table(eps), _table(sigma), _table(rc)
    f = np.zeros((n, 3)) if f is None else _f64(f).copy()
    maxrows = (nsteps // thermo_every + 2) if thermo_every > 0 else 1
    th = np.zeros((maxrows, 9))
    sk = -1.0 if skin is None else float(skin)
    rows = lib(timing).ref_md(n, _pd(x), _pd(v), _pd(f), _pi32(t), _pd(_f64(box)), eps.shape[0],
                        _pd(eps), _pd(sigma), _pd(rc), _pd(_f64(mass)), sk, float(dt),
                        int(step0), int(nsteps), int(rebuild_every), int(thermo_every),
                        int(setup), _pd(th))
    return x, v, f, th[:rows]


def equilibrate(x, v, types, box, eps, sigma, rc, mass, dt, nsteps, temperature, skin,
                rebuild_every=20):
    """Velocity-Verlet run from a fresh set-up over a Verlet list (cutoff rc +
    skin, rebuilt every rebuild_every steps) with the velocities rescaled to
    the kinetic temperature `temperature` after every step: the equilibration
    of a freshly placed liquid (input preparation).  Returns (x, v) copies,
    positions wrapped at the last rebuild."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    n = x.shape[0]
    t = _types(types, n)
    eps, sigma, rc = _table(eps), _table(sigma), _table(rc)
    f = np.zeros((n, 3))
    lib().ref_md_rescale(n, _pd(x), _pd(v), _pd(f), _pi32(t), _pd(_f64(box)), eps.shape[0],
                         _pd(eps), _pd(sigma), _pd(rc), _pd(_f64(mass)), float(skin), float(dt),
                         int(nsteps), int(rebuild_every), float(temperature))
    return x, v
