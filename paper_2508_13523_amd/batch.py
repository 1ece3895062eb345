"""Torch-facing binding of the batch entry points of libljmd (many independent
periodic systems in one set of launches): argument checks and marshalling
only, as in api.py."""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib as L
from .api import (LJParams, NeighborList, _need, _ptr, _stream, default_capacity, get_status,
                  thermo_rows)


class Batch:
    """nrep systems: system r owns atoms offsets[r] .. offsets[r+1]-1 and has
    box boxes[r].  Holds the host copies, the device copies and the C struct."""

    def __init__(self, offsets, boxes, device="cuda", tile_atoms: int = 0):
        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64).reshape(-1))
        self.boxes = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(-1, 3))
        if self.offsets.shape[0] != self.boxes.shape[0] + 1:
            raise ValueError("offsets must have one more entry than boxes")
        self.d_offsets = torch.as_tensor(self.offsets, device=device)
        self.d_boxes = torch.as_tensor(self.boxes, device=device)
        s = L.Batch()
        s.nrep = int(self.boxes.shape[0])
        s.tile_atoms = int(tile_atoms)
        s.offsets = self.offsets.ctypes.data
        s.boxes = self.boxes.ctypes.data
        s.d_offsets = self.d_offsets.data_ptr()
        s.d_boxes = self.d_boxes.data_ptr()
        self._c = s

    @classmethod
    def from_sizes(cls, sizes, boxes, device="cuda") -> "Batch":
        off = np.zeros(len(sizes) + 1, dtype=np.int64)
        np.cumsum(np.asarray(sizes, dtype=np.int64), out=off[1:])
        return cls(off, boxes, device)

    def c(self) -> L.Batch:
        return self._c

    @property
    def tile_atoms(self) -> int:
        """Home atoms per tile of the batch's tiled lists (0: the default);
        a list is read only with the value it was built with."""
        return int(self._c.tile_atoms)

    @tile_atoms.setter
    def tile_atoms(self, value: int) -> None:
        self._c.tile_atoms = int(value)

    @property
    def nrep(self) -> int:
        return int(self.boxes.shape[0])

    @property
    def n(self) -> int:
        return int(self.offsets[-1])

    def system(self, r: int) -> slice:
        return slice(int(self.offsets[r]), int(self.offsets[r + 1]))


def workspace_bytes(batch: Batch, params: LJParams) -> int:
    p = params.to_c()
    nbytes = L.load().ljmd_batch_workspace_bytes(ctypes.byref(batch.c()), ctypes.byref(p), 0)
    if nbytes == 0:
        code = L.load().ljmd_batch_nl_build(None, None, ctypes.byref(batch.c()), ctypes.byref(p),
                                            None, None, 0, None)
        raise L.LjmdError(code, "ljmd_batch_workspace_bytes")
    return int(nbytes)


def workspace(batch: Batch, params: LJParams, device="cuda") -> torch.Tensor:
    return torch.empty(max(workspace_bytes(batch, params), 256), dtype=torch.uint8,
                       device=device)


def neighbor_list(batch: Batch, params: LJParams, cap: int, device="cuda",
                  track_displacement: bool = True, global_format: bool = False) -> NeighborList:
    """A full list for the batch: tiled (default) or, with global_format, rows by
    batch-wide atom index.  Its export() goes through ljmd_batch_nl_export."""
    lib = L.load()
    p = params.to_c()
    aux_bytes = lib.ljmd_batch_aux_bytes(ctypes.byref(batch.c()), ctypes.byref(p))
    if aux_bytes == 0:
        workspace_bytes(batch, params)  # raises with the validation error
    nl = NeighborList.__new__(NeighborList)
    n = batch.n
    nl.n, nl.mode, nl.cap = n, L.FULL, int(cap)
    entries = lib.ljmd_nlist_entries(n, nl.cap)
    nl.numneigh = torch.zeros(max(n, 1), dtype=torch.int32, device=device)
    nl.neigh = torch.zeros(max(entries, 1), dtype=torch.int32, device=device)
    nl.status = torch.zeros(L.STATUS_WORDS, dtype=torch.int32, device=device)
    nl.xref = (torch.zeros((max(n, 1), 3), dtype=torch.float64, device=device)
               if track_displacement else None)
    nl.aux = torch.zeros(max(int(aux_bytes), 256), dtype=torch.uint8, device=device)
    s = L.NList()
    s.n, s.mode, s.cap = n, L.FULL, nl.cap
    s.numneigh = nl.numneigh.data_ptr()
    s.neigh = nl.neigh.data_ptr()
    s.status = nl.status.data_ptr()
    s.xref = nl.xref.data_ptr() if nl.xref is not None else None
    s.aux = nl.aux.data_ptr()
    s.aux_bytes = nl.aux.numel()
    s.flags = L.NL_GLOBAL if global_format else 0
    s.format = -1
    nl._c = s
    nl._batch = (batch, params)
    return nl


def nl_build(x, types, batch: Batch, params: LJParams, nl: NeighborList, ws=None):
    """ljmd_batch_nl_build (wraps x into each system's box in place)."""
    n = batch.n
    _need(x, "x", torch.float64, (n, 3))
    t = _need(types, "types", torch.int32, (n,)) if types is not None else None
    ws = workspace(batch, params, x.device) if ws is None else ws
    p = params.to_c()
    L.check(L.load().ljmd_batch_nl_build(_ptr(x), _ptr(t), ctypes.byref(batch.c()),
                                         ctypes.byref(p), ctypes.byref(nl.c()), _ptr(ws),
                                         ws.numel(), _stream()), "ljmd_batch_nl_build")
    return nl


def build_list(x, types, batch: Batch, params: LJParams, cap: Optional[int] = None, ws=None,
               track_displacement: bool = True, global_format: bool = False) -> NeighborList:
    """Allocate and build, growing the capacity until no row overflows
    (synchronizes)."""
    if cap is None:
        cap = max(default_capacity(params, batch.boxes[r], batch.offsets[r + 1] -
                                   batch.offsets[r]) for r in range(batch.nrep))
    while True:
        nl = neighbor_list(batch, params, cap, x.device, track_displacement, global_format)
        nl_build(x, types, batch, params, nl, ws)
        st = get_status(nl)
        if not st[L.ST_OVERFLOW]:
            return nl
        cap = int(st[L.ST_NEED]) + 8


def lj_forces(x, types, batch: Batch, params: LJParams, nl: NeighborList, mixed=False,
              ev=False, f=None, ws=None):
    """ljmd_batch_lj_forces: (f [n,3], ev [nrep,7] or None)."""
    n = batch.n
    _need(x, "x", torch.float64, (n, 3))
    t = _need(types, "types", torch.int32, (n,)) if types is not None else None
    f = torch.empty((n, 3), dtype=torch.float64, device=x.device) if f is None else \
        _need(f, "f", torch.float64, (n, 3))
    evt = torch.zeros((batch.nrep, 7), dtype=torch.float64, device=x.device) if ev else None
    ws = workspace(batch, params, x.device) if ws is None else ws
    flags = (L.PREC_MIXED if mixed else 0) | (L.EV if ev else 0)
    p = params.to_c()
    L.check(L.load().ljmd_batch_lj_forces(_ptr(x), _ptr(t), ctypes.byref(batch.c()),
                                          ctypes.byref(p), ctypes.byref(nl.c()), flags, _ptr(f),
                                          _ptr(evt), _ptr(ws), ws.numel(), _stream()),
            "ljmd_batch_lj_forces")
    return f, evt


def lj_backward(x, types, batch: Batch, params: LJParams, nl: NeighborList, gF, ws=None,
                gx=None, geps=None, gsig=None):
    """ljmd_batch_lj_backward: (gx [n,3], geps [T,T], gsig [T,T]), the
    parameter gradients summed over the systems."""
    n, T = batch.n, params.ntypes
    _need(x, "x", torch.float64, (n, 3))
    _need(gF, "gF", torch.float64, (n, 3))
    t = _need(types, "types", torch.int32, (n,)) if types is not None else None
    gx = torch.empty((n, 3), dtype=torch.float64, device=x.device) if gx is None else gx
    geps = torch.zeros((T, T), dtype=torch.float64, device=x.device) if geps is None else geps
    gsig = torch.zeros((T, T), dtype=torch.float64, device=x.device) if gsig is None else gsig
    ws = workspace(batch, params, x.device) if ws is None else ws
    p = params.to_c()
    L.check(L.load().ljmd_batch_lj_backward(_ptr(x), _ptr(t), ctypes.byref(batch.c()),
                                            ctypes.byref(p), ctypes.byref(nl.c()), _ptr(gF), 0,
                                            _ptr(gx), _ptr(geps), _ptr(gsig), _ptr(ws),
                                            ws.numel(), _stream()), "ljmd_batch_lj_backward")
    return gx, geps, gsig


def fm_grad(x, types, batch: Batch, params: LJParams, nl: NeighborList, f_target, weight=None,
            mixed: bool = False, f=None, ws=None, gx=None, geps=None, gsig=None):
    """ljmd_batch_fm_grad: the force-matching gradient of all systems in one
    call (loss sum_r (w_r/2) sum_i |F_i - f_target_i|^2, w_r = 2/N_r by
    default): (gx [n,3], geps [T,T], gsig [T,T]); f, if given, receives F."""
    n, T = batch.n, params.ntypes
    _need(x, "x", torch.float64, (n, 3))
    _need(f_target, "f_target", torch.float64, (n, 3))
    if weight is not None:
        _need(weight, "weight", torch.float64, (batch.nrep,))
    if f is not None:
        _need(f, "f", torch.float64, (n, 3))
    t = _need(types, "types", torch.int32, (n,)) if types is not None else None
    gx = torch.empty((n, 3), dtype=torch.float64, device=x.device) if gx is None else gx
    geps = torch.zeros((T, T), dtype=torch.float64, device=x.device) if geps is None else geps
    gsig = torch.zeros((T, T), dtype=torch.float64, device=x.device) if gsig is None else gsig
    ws = workspace(batch, params, x.device) if ws is None else ws
    p = params.to_c()
    L.check(L.load().ljmd_batch_fm_grad(_ptr(x), _ptr(t), ctypes.byref(batch.c()),
                                        ctypes.byref(p), ctypes.byref(nl.c()), _ptr(f_target),
                                        _ptr(weight), L.PREC_MIXED if mixed else 0, _ptr(f),
                                        _ptr(gx), _ptr(geps), _ptr(gsig), _ptr(ws), ws.numel(),
                                        _stream()), "ljmd_batch_fm_grad")
    return gx, geps, gsig


def md_step(x, v, f, types, batch: Batch, params: LJParams, nl: NeighborList, dt: float,
            nsteps: int, step0: int = 0, rebuild_every: int = 20, thermo_every: int = 0,
            setup: bool = False, mixed: bool = False, sync_check: bool = False,
            sort: bool = False, ids=None, ws=None, thermo=None, separate_kick: bool = False):
    """ljmd_batch_md_step: advances every system in place; returns the thermo
    rows [rows, nrep, 9].  separate_kick runs the velocity-Verlet updates as
    kernels of their own instead of in the tiled gather's epilogue."""
    n = batch.n
    for name, a in (("x", x), ("v", v), ("f", f)):
        _need(a, name, torch.float64, (n, 3))
    t = _need(types, "types", torch.int32, (n,)) if types is not None else None
    if ids is not None:
        _need(ids, "ids", torch.int32, (n,))
    rows = thermo_rows(step0, nsteps, thermo_every, setup)
    if thermo is None:
        thermo = torch.zeros((max(rows, 1), batch.nrep, 9), dtype=torch.float64,
                             device=x.device)
    ws = workspace(batch, params, x.device) if ws is None else ws
    flags = ((L.PREC_MIXED if mixed else 0) | (L.SETUP if setup else 0) |
             (L.SYNC_CHECK if sync_check else 0) | (L.SORT if sort else 0) |
             (L.SEPARATE_KICK if separate_kick else 0))
    p = params.to_c()
    L.check(L.load().ljmd_batch_md_step(_ptr(x), _ptr(v), _ptr(f), _ptr(t), _ptr(ids),
                                        ctypes.byref(batch.c()), ctypes.byref(p),
                                        ctypes.byref(nl.c()), float(dt), int(step0),
                                        int(nsteps), int(rebuild_every), int(thermo_every),
                                        flags, _ptr(thermo), _ptr(ws), ws.numel(), _stream()),
            "ljmd_batch_md_step")
    return thermo[:rows]


TILE_SEARCH = (150, 200, 300, 450, 600)  # the tile targets ljmd_batch_autotune tries


def autotune(x, types, batch: Batch, params: LJParams, nl: NeighborList, mixed=False, f=None,
             ws=None, tiles: bool = False, for_md: bool = False) -> tuple:
    """ljmd_batch_autotune: (lanes_per_atom, block, persistent, tile_atoms) of
    the fastest force variant, kept for later calls of this batch class
    (synchronizes).  With tiles=True the tile target is searched as well: nl
    is rebuilt for the chosen one and batch.tile_atoms is set to it; the
    tiling is weighed for the force-matching gradient, or with for_md=True
    for the MD step."""
    n = batch.n
    _need(x, "x", torch.float64, (n, 3))
    t = _need(types, "types", torch.int32, (n,)) if types is not None else None
    f = torch.empty((n, 3), dtype=torch.float64, device=x.device) if f is None else f
    if ws is None:
        # room for every tile target the search tries (smaller tiles, more
        # per-tile partial sums)
        nbytes = workspace_bytes(batch, params)
        if tiles:
            for target in TILE_SEARCH:
                probe = Batch(batch.offsets, batch.boxes, x.device, tile_atoms=target)
                nbytes = max(nbytes, workspace_bytes(probe, params))
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=x.device)
    best = L.BatchTuning()
    p = params.to_c()
    flags = ((L.PREC_MIXED if mixed else 0) | (L.TUNE_TILES if tiles else 0) |
             (L.TUNE_MD if for_md else 0))
    L.check(L.load().ljmd_batch_autotune(_ptr(x), _ptr(t), ctypes.byref(batch.c()),
                                         ctypes.byref(p), ctypes.byref(nl.c()), flags, _ptr(f),
                                         _ptr(ws), ws.numel(), _stream(), ctypes.byref(best)),
            "ljmd_batch_autotune")
    if tiles:
        batch.tile_atoms = int(best.tile_atoms)
    return (int(best.lanes_per_atom), int(best.block), int(best.persistent),
            int(best.tile_atoms))


def set_tuning(batch: Batch, params: LJParams, tuning, mixed=False) -> None:
    """ljmd_batch_set_tuning: force (lanes_per_atom, block, persistent), or
    clear with None."""
    p = params.to_c()
    tp = None
    if tuning is not None:
        tp = L.BatchTuning()
        tp.lanes_per_atom, tp.block, tp.persistent = (int(v) for v in tuning[:3])
        tp = ctypes.byref(tp)
    L.check(L.load().ljmd_batch_set_tuning(ctypes.byref(batch.c()), ctypes.byref(p),
                                           L.PREC_MIXED if mixed else 0, tp),
            "ljmd_batch_set_tuning")
