"""Torch-facing binding of libljmd: argument checks and marshalling only.

Every function takes CUDA (HIP) tensors, passes their device pointers and
torch's current stream to the matching C entry point of include/ljmd.h, and
raises LjmdError on a negative return code.  No arithmetic of the method
happens here.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


# ---------------------------------------------------------------- parameters


@dataclasses.dataclass
class LJParams:
    """Per-type-pair tables (ntypes x ntypes, symmetric), skin and masses."""

    eps: np.ndarray
    sigma: np.ndarray
    rc: np.ndarray
    skin: float = 0.3
    mass: Optional[np.ndarray] = None

    def __post_init__(self):
        self.eps = np.atleast_2d(np.asarray(self.eps, dtype=np.float64))
        self.sigma = np.atleast_2d(np.asarray(self.sigma, dtype=np.float64))
        self.rc = np.atleast_2d(np.asarray(self.rc, dtype=np.float64))
        if self.mass is None:
            self.mass = np.ones(self.ntypes)
        self.mass = np.asarray(self.mass, dtype=np.float64).reshape(-1)

    @property
    def ntypes(self) -> int:
        return int(self.eps.shape[0])

    @property
    def max_neighbor_cutoff(self) -> float:
        return float(self.rc.max() + self.skin)

    def to_c(self) -> L.Params:
        p = L.Params()
        T = self.ntypes
        p.ntypes = T
        if T > L.MAX_TYPES or self.sigma.shape != (T, T) or self.rc.shape != (T, T):
            # let the library report the error for out-of-range type counts
            T = min(T, L.MAX_TYPES)
        for a in range(T):
            for b in range(T):
                p.eps[a][b] = float(self.eps[a, b])
                p.sigma[a][b] = float(self.sigma[a, b])
                p.rc[a][b] = float(self.rc[a, b])
            p.mass[a] = float(self.mass[a]) if a < self.mass.shape[0] else 0.0
        p.skin = float(self.skin)
        return p

    @staticmethod
    def from_system(s) -> "LJParams":
        return LJParams(eps=s.eps, sigma=s.sigma, rc=s.rc, skin=s.skin, mass=s.mass)


def c_box(box: Sequence[float]) -> L.Box:
    b = L.Box()
    vals = [float(v) for v in np.asarray(box, dtype=np.float64).reshape(-1)]
    if len(vals) != 3:
        raise ValueError("box must have 3 lengths")
    b.len[0], b.len[1], b.len[2] = vals
    return b


# ---------------------------------------------------------------- helpers


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(t: torch.Tensor, name: str, dtype, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _types(types, n, params: LJParams):
    if types is None:
        if params.ntypes > 1:
            raise ValueError("types are required when ntypes > 1")
        return None
    return _need(types, "types", torch.int32, (n,))


# ---------------------------------------------------------------- objects


class NeighborList:
    """Device storage of an ljmd_nlist: numneigh [n], neigh (entries in the
    format the build picks, held in an int32 tensor), status [4], xref [n, 3]
    and aux (the cell order the list was built in).  The host struct is kept
    alive here so the fields the build writes (format, tile, cells) persist."""

    def __init__(self, n: int, cap: int, box, params: "LJParams", mode: str = "full",
                 device="cuda", track_displacement: bool = True, global_format: bool = False):
        self.n = int(n)
        self.mode = L.HALF if mode == "half" else L.FULL
        self.cap = int(cap)
        lib = L.load()
        entries = lib.ljmd_nlist_entries(self.n, self.cap)
        b, p = c_box(box), params.to_c()
        aux_bytes = lib.ljmd_nlist_aux_bytes(self.n, ctypes.byref(b), ctypes.byref(p))
        if aux_bytes == 0:
            workspace_bytes(self.n, box, params)  # raises with the validation error
        self.numneigh = torch.zeros(max(self.n, 1), dtype=torch.int32, device=device)
        self.neigh = torch.zeros(max(entries, 1), dtype=torch.int32, device=device)
        self.status = torch.zeros(L.STATUS_WORDS, dtype=torch.int32, device=device)
        self.xref = (torch.zeros((max(self.n, 1), 3), dtype=torch.float64, device=device)
                     if track_displacement else None)
        self.aux = torch.zeros(max(int(aux_bytes), 256), dtype=torch.uint8, device=device)
        s = L.NList()
        s.n = self.n
        s.mode = self.mode
        s.cap = self.cap
        s.numneigh = self.numneigh.data_ptr()
        s.neigh = self.neigh.data_ptr()
        s.status = self.status.data_ptr()
        s.xref = self.xref.data_ptr() if self.xref is not None else None
        s.aux = self.aux.data_ptr()
        s.aux_bytes = self.aux.numel()
        s.flags = L.NL_GLOBAL if global_format else 0
        s.format = -1
        self._c = s

    def c(self) -> L.NList:
        return self._c

    @property
    def format(self) -> str:
        return {L.FMT_GLOBAL: "global", L.FMT_TILED: "tiled"}.get(self._c.format, "unbuilt")

    @property
    def tile(self) -> tuple:
        """Cells per workgroup along x, y, z recorded by the last build."""
        return tuple(int(v) for v in self._c.tile)

    def status_host(self) -> np.ndarray:
        return get_status(self)

    def export(self):
        """ljmd_nl_export: (entries, counts) on the GPU in the global format,
        rows by atom index."""
        entries = L.load().ljmd_nlist_entries(self.n, self.cap)
        out = torch.zeros(max(entries, 1), dtype=torch.int32, device=self.neigh.device)
        counts = torch.zeros(max(self.n, 1), dtype=torch.int32, device=self.neigh.device)
        batch = getattr(self, "_batch", None)
        if batch is not None:  # a batch list: exported through its batch
            from . import batch as B
            bt, prm = batch
            ws = B.workspace(bt, prm, self.neigh.device)
            L.check(L.load().ljmd_batch_nl_export(ctypes.byref(self._c), ctypes.byref(bt.c()),
                                                  ctypes.byref(prm.to_c()), _ptr(out),
                                                  _ptr(counts), _ptr(ws), ws.numel(), _stream()),
                    "ljmd_batch_nl_export")
            return out, counts
        L.check(L.load().ljmd_nl_export(ctypes.byref(self._c), _ptr(out), _ptr(counts),
                                        _stream()), "ljmd_nl_export")
        return out, counts

    def export_indices(self):
        """ljmd_nl_export_indices: (idx [cap, n] int32, counts [n] int32) on the
        GPU, entry k of atom i's row at idx[k, i]; entries beyond counts[i]
        are -1."""
        out = torch.full((self.cap, max(self.n, 1)), -1, dtype=torch.int32,
                         device=self.neigh.device)
        counts = torch.zeros(max(self.n, 1), dtype=torch.int32, device=self.neigh.device)
        L.check(L.load().ljmd_nl_export_indices(ctypes.byref(self._c), _ptr(out), _ptr(counts),
                                                _stream()), "ljmd_nl_export_indices")
        return out[:, : self.n], counts[: self.n]

    def rows_csr(self, rows):
        """Selected rows only (gathered on the GPU): (counts, offsets, idx, codes),
        each row sorted by index."""
        out, cnts = self.export()
        rows_t = torch.as_tensor(np.asarray(rows, dtype=np.int64), device=out.device)
        cnt = cnts[rows_t].to(torch.int64)
        k = torch.arange(self.cap, device=out.device, dtype=torch.int64)
        base = (rows_t >> 6) * (self.cap * 64) + (rows_t & 63)
        pos = base[:, None] + k[None, :] * 64
        vals = out[pos].cpu().numpy().view(np.uint32)
        counts = cnt.cpu().numpy()
        mask = np.arange(self.cap)[None, :] < counts[:, None]
        v = vals[mask]
        idx = (v & np.uint32((1 << 26) - 1)).astype(np.int32)
        codes = (v >> np.uint32(26)).astype(np.int32)
        offsets = np.zeros(len(counts) + 1, dtype=np.int64)
        np.cumsum(counts, out=offsets[1:])
        order = np.lexsort((idx, np.repeat(np.arange(len(counts)), counts)))
        return counts, offsets, idx[order], codes[order]

    def to_csr(self):
        """All rows on the host by atom index: (counts, offsets, idx, codes), each
        row sorted by index; codes are the 6-bit image codes of the entries."""
        n, cap = self.n, self.cap
        out, cnts = self.export()
        counts = cnts[:n].cpu().numpy().astype(np.int64)
        raw = out.cpu().numpy().view(np.uint32)
        nb = (n + 63) // 64
        tiles = raw[: nb * 64 * cap].reshape(nb, cap, 64)
        rows = tiles.transpose(0, 2, 1).reshape(nb * 64, cap)[:n]
        mask = np.arange(cap)[None, :] < counts[:, None]
        vals = rows[mask]
        idx = (vals & np.uint32((1 << 26) - 1)).astype(np.int32)
        codes = (vals >> np.uint32(26)).astype(np.int32)
        offsets = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(counts, out=offsets[1:])
        order = np.lexsort((idx, np.repeat(np.arange(n), counts)))
        return counts, offsets, idx[order], codes[order]


_WS_CACHE: dict = {}


def workspace(n: int, box, params: LJParams, device="cuda") -> torch.Tensor:
    """Scratch buffer of ljmd_workspace_bytes() bytes (cached per size)."""
    nbytes = workspace_bytes(n, box, params)
    key = (str(device), torch.cuda.current_device())
    ws = _WS_CACHE.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _WS_CACHE[key] = ws
    return ws


def workspace_bytes(n: int, box, params: LJParams) -> int:
    b, p = c_box(box), params.to_c()
    nbytes = L.load().ljmd_workspace_bytes(int(n), ctypes.byref(b), ctypes.byref(p), 0)
    if nbytes == 0:
        # reproduce the validation error with a call that reports it
        code = L.load().ljmd_nl_build(None, None, int(n), ctypes.byref(b), ctypes.byref(p),
                                      None, None, 0, None)
        raise L.LjmdError(code, "ljmd_workspace_bytes")
    return int(nbytes)


def default_capacity(params: LJParams, box, n: int) -> int:
    """Generous capacity guess: 1.4x the ideal-gas count within the largest
    neighbor cutoff, plus 32."""
    vol = float(np.prod(np.asarray(box, dtype=np.float64)))
    rho = n / vol if vol > 0 else 0.0
    r = params.max_neighbor_cutoff
    return int(1.4 * rho * 4.0 / 3.0 * math.pi * r ** 3) + 32


# ---------------------------------------------------------------- entry points


def nl_build(x: torch.Tensor, types, box, params: LJParams, nl: NeighborList,
             ws: Optional[torch.Tensor] = None) -> NeighborList:
    """ljmd_nl_build: wraps x into the box in place and rebuilds nl."""
    n = nl.n
    _need(x, "x", torch.float64, (n, 3))
    t = _types(types, n, params)
    ws = workspace(n, box, params, x.device) if ws is None else ws
    b, p, s = c_box(box), params.to_c(), nl.c()
    L.check(L.load().ljmd_nl_build(_ptr(x), _ptr(t), n, ctypes.byref(b), ctypes.byref(p),
                                   ctypes.byref(s), _ptr(ws), ws.numel(), _stream()),
            "ljmd_nl_build")
    return nl


def build_list(x: torch.Tensor, types, box, params: LJParams, mode: str = "full",
               cap: Optional[int] = None, ws=None, track_displacement: bool = True,
               global_format: bool = False) -> NeighborList:
    """Allocate and build a list, growing the capacity until no row overflows
    and falling back to the global format if a stencil outgrows 16-bit slots
    (reads the status word, so it synchronizes)."""
    n = int(x.shape[0])
    cap = default_capacity(params, box, n) if cap is None else int(cap)
    while True:
        nl = NeighborList(n, cap, box, params, mode, x.device, track_displacement, global_format)
        nl_build(x, types, box, params, nl, ws)
        st = get_status(nl)
        if st[L.ST_OVERFLOW] & 2:
            global_format = True
            continue
        if not st[L.ST_OVERFLOW]:
            return nl
        cap = int(st[L.ST_NEED]) + 8


def lj_forces(x: torch.Tensor, types, box, params: LJParams, nl: NeighborList,
              mixed: bool = False, ev: bool = False, f: Optional[torch.Tensor] = None,
              ws: Optional[torch.Tensor] = None):
    """ljmd_lj_forces: returns (f [n,3], ev [7] or None) on the GPU."""
    n = nl.n
    _need(x, "x", torch.float64, (n, 3))
    t = _types(types, n, params)
    f = torch.empty((n, 3), dtype=torch.float64, device=x.device) if f is None else \
        _need(f, "f", torch.float64, (n, 3))
    evt = torch.zeros(7, dtype=torch.float64, device=x.device) if ev else None
    ws = workspace(n, box, params, x.device) if ws is None else ws
    flags = (L.PREC_MIXED if mixed else 0) | (L.EV if ev else 0)
    b, p, s = c_box(box), params.to_c(), nl.c()
    L.check(L.load().ljmd_lj_forces(_ptr(x), _ptr(t), n, ctypes.byref(b), ctypes.byref(p),
                                    ctypes.byref(s), flags, _ptr(f), _ptr(evt), _ptr(ws),
                                    ws.numel(), _stream()), "ljmd_lj_forces")
    return f, evt


def lj_backward(x: torch.Tensor, types, box, params: LJParams, nl: NeighborList,
                gF: torch.Tensor, ws: Optional[torch.Tensor] = None):
    """ljmd_lj_backward: returns (gx [n,3], geps [T,T], gsig [T,T]) on the GPU."""
    n = nl.n
    T = params.ntypes
    _need(x, "x", torch.float64, (n, 3))
    _need(gF, "gF", torch.float64, (n, 3))
    t = _types(types, n, params)
    gx = torch.empty((n, 3), dtype=torch.float64, device=x.device)
    geps = torch.empty((T, T), dtype=torch.float64, device=x.device)  # every entry written
    gsig = torch.empty((T, T), dtype=torch.float64, device=x.device)
    ws = workspace(n, box, params, x.device) if ws is None else ws
    b, p, s = c_box(box), params.to_c(), nl.c()
    L.check(L.load().ljmd_lj_backward(_ptr(x), _ptr(t), n, ctypes.byref(b), ctypes.byref(p),
                                      ctypes.byref(s), _ptr(gF), 0, _ptr(gx), _ptr(geps),
                                      _ptr(gsig), _ptr(ws), ws.numel(), _stream()),
            "ljmd_lj_backward")
    return gx, geps, gsig


def fm_grad(x: torch.Tensor, types, box, params: LJParams, nl: NeighborList,
            f_target: torch.Tensor, weight: Optional[torch.Tensor] = None, mixed: bool = False,
            f: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
            gx: Optional[torch.Tensor] = None):
    """ljmd_fm_grad: the force-matching gradient of L = (w/2) sum_i |F_i -
    f_target_i|^2 (w = 2/n by default: the mean over atoms) in one call:
    returns (gx [n,3], geps [T,T], gsig [T,T]); f, if given, receives F."""
    n = nl.n
    T = params.ntypes
    _need(x, "x", torch.float64, (n, 3))
    _need(f_target, "f_target", torch.float64, (n, 3))
    if weight is not None:
        _need(weight, "weight", torch.float64, (1,))
    if f is not None:
        _need(f, "f", torch.float64, (n, 3))
    t = _types(types, n, params)
    gx = torch.empty((n, 3), dtype=torch.float64, device=x.device) if gx is None else gx
    geps = torch.empty((T, T), dtype=torch.float64, device=x.device)
    gsig = torch.empty((T, T), dtype=torch.float64, device=x.device)
    ws = workspace(n, box, params, x.device) if ws is None else ws
    b, p, s = c_box(box), params.to_c(), nl.c()
    L.check(L.load().ljmd_fm_grad(_ptr(x), _ptr(t), n, ctypes.byref(b), ctypes.byref(p),
                                  ctypes.byref(s), _ptr(f_target), _ptr(weight),
                                  L.PREC_MIXED if mixed else 0, _ptr(f), _ptr(gx), _ptr(geps),
                                  _ptr(gsig), _ptr(ws), ws.numel(), _stream()), "ljmd_fm_grad")
    return gx, geps, gsig


def lj_backward_noalloc(x: torch.Tensor, types, box, params: LJParams, nl: NeighborList,
                        gF: torch.Tensor, gx: torch.Tensor, geps: torch.Tensor,
                        gsig: torch.Tensor):
    """ljmd_lj_backward_noalloc: ljmd_lj_backward into caller-given outputs
    (gx [n,3], geps and gsig [T,T], float64 on the GPU) with no workspace:
    the library's static device scratch holds the partial sums."""
    n = nl.n
    T = params.ntypes
    _need(x, "x", torch.float64, (n, 3))
    _need(gF, "gF", torch.float64, (n, 3))
    _need(gx, "gx", torch.float64, (n, 3))
    _need(geps, "geps", torch.float64, (T, T))
    _need(gsig, "gsig", torch.float64, (T, T))
    t = _types(types, n, params)
    b, p, s = c_box(box), params.to_c(), nl.c()
    L.check(L.load().ljmd_lj_backward_noalloc(_ptr(x), _ptr(t), n, ctypes.byref(b),
                                              ctypes.byref(p), ctypes.byref(s), _ptr(gF), 0,
                                              _ptr(gx), _ptr(geps), _ptr(gsig), _stream()),
            "ljmd_lj_backward_noalloc")
    return gx, geps, gsig


def thermo_rows(step0: int, nsteps: int, thermo_every: int, setup: bool) -> int:
    if thermo_every <= 0:
        return 0
    first = step0 if setup else step0 + 1
    last = step0 + nsteps
    if last < first:
        return 0
    return last // thermo_every - (first - 1) // thermo_every


def md_step(x, v, f, types, box, params: LJParams, nl: NeighborList, dt: float, nsteps: int,
            step0: int = 0, rebuild_every: int = 20, thermo_every: int = 0, setup: bool = False,
            mixed: bool = False, sync_check: bool = False, sort: bool = False, ids=None, ws=None,
            thermo=None, separate_kick: bool = False):
    """ljmd_md_step: advances x, v, f (and nl) in place; returns the thermo
    rows [rows, 9] (g, E, KE, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz) on the GPU.  With
    sort=True atoms are reordered into cell order at every build; types and
    ids (int32 [n], optional) are permuted with them.  separate_kick=True
    keeps the velocity-Verlet updates out of the force kernel."""
    n = nl.n
    for name, t in (("x", x), ("v", v), ("f", f)):
        _need(t, name, torch.float64, (n, 3))
    t = _types(types, n, params)
    if ids is not None:
        _need(ids, "ids", torch.int32, (n,))
    rows = thermo_rows(step0, nsteps, thermo_every, setup)
    if thermo is None:
        thermo = torch.zeros((max(rows, 1), 9), dtype=torch.float64, device=x.device)
    ws = workspace(n, box, params, x.device) if ws is None else ws
    flags = ((L.PREC_MIXED if mixed else 0) | (L.SETUP if setup else 0) |
             (L.SYNC_CHECK if sync_check else 0) | (L.SORT if sort else 0) |
             (L.SEPARATE_KICK if separate_kick else 0))
    b, p, s = c_box(box), params.to_c(), nl.c()
    L.check(L.load().ljmd_md_step(_ptr(x), _ptr(v), _ptr(f), _ptr(t), _ptr(ids), n, ctypes.byref(b),
                                  ctypes.byref(p), ctypes.byref(s), float(dt), int(step0),
                                  int(nsteps), int(rebuild_every), int(thermo_every), flags,
                                  _ptr(thermo), _ptr(ws), ws.numel(), _stream()),
            "ljmd_md_step")
    return thermo[:rows]


def get_status(nl: NeighborList) -> np.ndarray:
    """ljmd_get_status: the status words on the host (synchronizes)."""
    out = (ctypes.c_int32 * L.STATUS_WORDS)()
    s = nl.c()
    L.check(L.load().ljmd_get_status(ctypes.byref(s), out, _stream()), "ljmd_get_status")
    return np.array(list(out), dtype=np.int64)


def strerror(code: int) -> str:
    return L.strerror(code)


def profile_enable(on: bool = True) -> None:
    """ljmd_profile_enable: bracket every phase with HIP events."""
    L.check(L.load().ljmd_profile_enable(1 if on else 0), "ljmd_profile_enable")


def profile_read() -> dict:
    """ljmd_profile_read: {phase: (total ms, instances)} since the last read."""
    ms = (ctypes.c_double * len(L.PHASES))()
    cnt = (ctypes.c_int64 * len(L.PHASES))()
    L.check(L.load().ljmd_profile_read(ms, cnt), "ljmd_profile_read")
    return {name: (float(ms[k]), int(cnt[k])) for k, name in enumerate(L.PHASES)}


def set_gather_lanes(lanes: int) -> None:
    """ljmd_set_gather_lanes: lanes (1, 2, 4, 8; 0 = automatic: per tile, or
    for the gather of large tiles from the tile size) sharing one atom's row
    in the tiled full-list force gather and adjoint."""
    L.check(L.load().ljmd_set_gather_lanes(int(lanes)), "ljmd_set_gather_lanes")


def get_gather_lanes() -> int:
    """ljmd_get_gather_lanes: the current setting (0: automatic)."""
    return int(L.load().ljmd_get_gather_lanes())


def nl_gather_lanes(nl: NeighborList, box, params: LJParams) -> int:
    """ljmd_nl_gather_lanes: lanes per atom the gather uses on this built list
    (0: chosen per tile)."""
    b, p, s = c_box(box), params.to_c(), nl.c()
    return L.check_value(L.load().ljmd_nl_gather_lanes(ctypes.byref(s), ctypes.byref(b),
                                                       ctypes.byref(p)), "ljmd_nl_gather_lanes")
