"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/ljmd.h declares, and rejects bad arguments with the
documented codes before touching the GPU."""
import ctypes

import numpy as np
import pytest

from paper_2508_13523_amd import _lib as L
from paper_2508_13523_amd import api, inputs


@pytest.fixture(scope="module")
def lib():
    import os
    if not os.path.exists(L.LIB_PATH):
        from paper_2508_13523_amd import build
        build.build()
    return L.load()


def cparams(ntypes=1, eps=1.0, sig=1.0, rc=2.5, skin=0.3):
    p = L.Params()
    p.ntypes = ntypes
    for a in range(min(ntypes, 4)):
        for b in range(min(ntypes, 4)):
            p.eps[a][b] = eps
            p.sigma[a][b] = sig
            p.rc[a][b] = rc
        p.mass[a] = 1.0
    p.skin = skin
    return p


def cbox(L_=10.0):
    b = L.Box()
    b.len[0] = b.len[1] = b.len[2] = L_
    return b


def test_exports_every_declared_symbol(lib):
    names = L.header_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.SIGNATURES)


def test_strerror_covers_codes(lib):
    for code in (L.OK, L.EINVAL, L.EBOX, L.EWORKSPACE, L.ENEIGH_OVERFLOW, L.ENOTSUP, L.EHIP,
                 L.ESCRATCH):
        assert L.strerror(code) and L.strerror(code) != "unknown error code"
    assert L.strerror(-99) == "unknown error code"


def test_nlist_entries(lib):
    # rows padded to 64 atoms, capacity rounded up to a multiple of 16
    assert lib.ljmd_nlist_entries(1, 12) == 64 * 16
    assert lib.ljmd_nlist_entries(64, 17) == 64 * 32
    assert lib.ljmd_nlist_entries(65, 3) == 128 * 16
    assert lib.ljmd_nlist_entries(65, 32) == 128 * 32
    assert lib.ljmd_nlist_entries(0, 3) == 0
    assert lib.ljmd_nlist_entries(5, 0) == 0


def test_workspace_bytes(lib):
    b, p = cbox(16.8), cparams()
    w1 = lib.ljmd_workspace_bytes(4000, ctypes.byref(b), ctypes.byref(p), 0)
    w2 = lib.ljmd_workspace_bytes(8000, ctypes.byref(b), ctypes.byref(p), 0)
    assert 0 < w1 < w2 and w1 % 256 == 0
    assert lib.ljmd_workspace_bytes(0, ctypes.byref(b), ctypes.byref(p), 0) > 0
    b2 = cbox(5.0)  # < 2 * 2.8
    assert lib.ljmd_workspace_bytes(10, ctypes.byref(b2), ctypes.byref(p), 0) == 0
    # aux: cell order (4 B per atom) and cell starts (4 B per cell + 1), 256-aligned
    a = lib.ljmd_nlist_aux_bytes(4000, ctypes.byref(b), ctypes.byref(p))
    assert a == 16000 + 256 - 16000 % 256 + ((126 * 4 + 255) // 256) * 256
    assert lib.ljmd_nlist_aux_bytes(10, ctypes.byref(b2), ctypes.byref(p)) == 0


def fake_nlist(n=10, mode=L.FULL, cap=8):
    """A list struct whose pointers are never dereferenced (validation only)."""
    nl = L.NList()
    nl.n, nl.mode, nl.cap = n, mode, cap
    nl.numneigh = nl.neigh = nl.status = nl.aux = 0x1000
    nl.aux_bytes = 1 << 30
    nl.format = L.FMT_GLOBAL
    return nl


def _build(lib, n=10, box=None, p=None, nl=None, ws_bytes=1 << 30, ws=0x1000):
    box = box or cbox()
    p = p or cparams()
    if nl is None:
        nl = fake_nlist(n)
    return lib.ljmd_nl_build(ctypes.c_void_p(0x1000), None, n, ctypes.byref(box), ctypes.byref(p),
                             ctypes.byref(nl), ctypes.c_void_p(ws), ws_bytes, None)


def test_validation_codes(lib):
    assert _build(lib, box=cbox(5.59)) == L.EBOX
    assert _build(lib, p=cparams(ntypes=0)) == L.EINVAL
    assert _build(lib, p=cparams(ntypes=5)) == L.ENOTSUP
    p = cparams(ntypes=2)
    p.eps[0][1] = 1.5  # asymmetric
    assert _build(lib, p=p) == L.EINVAL
    assert _build(lib, p=cparams(eps=-1.0)) == L.EINVAL
    assert _build(lib, p=cparams(skin=-0.1)) == L.EINVAL
    assert _build(lib, p=cparams(rc=float("nan"))) == L.EINVAL
    assert _build(lib, box=cbox(2.0e9)) == L.EINVAL
    # a cell grid whose counts would not fit the int32 cell tables: rejected
    # before any conversion (1e8 / (1e-6 + 0) = 1e14 cells per dimension)
    assert _build(lib, box=cbox(1.0e8), p=cparams(rc=1e-6, skin=0.0)) == L.ENOTSUP
    # 1,400 cells per dimension fit one dimension but not the whole table
    assert _build(lib, box=cbox(1400.0), p=cparams(rc=0.7, skin=0.3)) == L.ENOTSUP
    assert _build(lib, n=-1) == L.EINVAL
    assert _build(lib, n=1 << 26) == L.ENOTSUP
    assert _build(lib, ws_bytes=16) == L.EWORKSPACE
    assert _build(lib, ws=0x1008) == L.EINVAL  # workspace not 256-byte aligned
    nl = fake_nlist(11)  # n mismatch
    assert _build(lib, nl=nl) == L.EINVAL
    nl = fake_nlist(10)
    nl.aux_bytes = 16  # aux smaller than ljmd_nlist_aux_bytes
    assert _build(lib, nl=nl) == L.EINVAL
    nl = fake_nlist(10)
    nl.aux = None
    assert _build(lib, nl=nl) == L.EINVAL
    nl.n, nl.cap = 10, 0
    assert _build(lib, nl=nl) == L.EINVAL
    nl.cap, nl.mode = 8, 7
    assert _build(lib, nl=nl) == L.EINVAL
    # ntypes > 1 requires the type array
    p2 = cparams(ntypes=2)
    assert _build(lib, p=p2) == L.EINVAL


def test_backward_and_md_validation(lib):
    b, p = cbox(), cparams()
    nl = fake_nlist(10, L.HALF)
    d = ctypes.c_void_p(0x1000)
    rc = lib.ljmd_lj_backward(d, None, 10, ctypes.byref(b), ctypes.byref(p), ctypes.byref(nl), d,
                              0, d, None, None, d, 1 << 30, None)
    assert rc == L.ENOTSUP  # half list
    nl.mode = L.FULL
    rc = lib.ljmd_lj_backward(d, None, 10, ctypes.byref(b), ctypes.byref(p), ctypes.byref(nl), d,
                              L.PREC_MIXED, d, None, None, d, 1 << 30, None)
    assert rc == L.ENOTSUP  # FP64 only
    # forces on a list that was never built, or built for another cell grid
    for fmt, cells in [(-1, (3, 3, 3)), (L.FMT_TILED, (3, 3, 3)), (L.FMT_GLOBAL, (9, 3, 3))]:
        nl.format = fmt
        nl.ncell[0], nl.ncell[1], nl.ncell[2] = cells
        rc = lib.ljmd_lj_forces(d, None, 10, ctypes.byref(b), ctypes.byref(p), ctypes.byref(nl),
                                0, d, None, d, 1 << 30, None)
        assert rc == L.EINVAL, (fmt, cells)
    nl.format = -1
    assert lib.ljmd_nl_export(ctypes.byref(nl), d, d, None) == L.EINVAL
    for dt, nsteps, reb, th in [(0.0, 1, 20, 0), (-1.0, 1, 20, 0), (0.005, -1, 20, 0),
                                (0.005, 1, 0, 0), (0.005, 1, 20, -1), (0.005, 1, 20, 5)]:
        rc = lib.ljmd_md_step(d, d, d, None, None, 10, ctypes.byref(b), ctypes.byref(p),
                              ctypes.byref(nl), dt, 0, nsteps, reb, th, 0, None, d, 1 << 30, None)
        assert rc == L.EINVAL, (dt, nsteps, reb, th)
    p.mass[0] = 0.0
    rc = lib.ljmd_md_step(d, d, d, None, None, 10, ctypes.byref(b), ctypes.byref(p), ctypes.byref(nl),
                          0.005, 0, 1, 20, 0, 0, None, d, 1 << 30, None)
    assert rc == L.EINVAL


def test_backward_noalloc_validation(lib):
    """The allocation-free adjoint checks its arguments like ljmd_lj_backward,
    and rejects a problem needing more partial-sum rows than its static
    scratch holds with LJMD_ESCRATCH, before any HIP call."""
    b, p = cbox(), cparams()
    d = ctypes.c_void_p(0x1000)
    nl = fake_nlist(10, L.HALF)
    rc = lib.ljmd_lj_backward_noalloc(d, None, 10, ctypes.byref(b), ctypes.byref(p),
                                      ctypes.byref(nl), d, 0, d, None, None, None)
    assert rc == L.ENOTSUP  # half list
    nl.mode = L.FULL
    rc = lib.ljmd_lj_backward_noalloc(d, None, 10, ctypes.byref(b), ctypes.byref(p),
                                      ctypes.byref(nl), d, L.PREC_MIXED, d, None, None, None)
    assert rc == L.ENOTSUP  # FP64 only
    # a global-format list of 256 * LJMD_NOALLOC_MAX_BLOCKS + 1 atoms in a box of
    # 3 x 3 x 3 cells (strips of one cell at this density): one row too many
    n = 256 * L.NOALLOC_MAX_BLOCKS + 1
    nl = fake_nlist(n)
    nl.format = L.FMT_GLOBAL
    for k in range(3):
        nl.ncell[k] = 3
        nl.tile[k] = 1
    rc = lib.ljmd_lj_backward_noalloc(d, None, n, ctypes.byref(b), ctypes.byref(p),
                                      ctypes.byref(nl), d, 0, d, None, None, None)
    assert rc == L.ESCRATCH
    assert "LJMD_NOALLOC_MAX_BLOCKS" in L.strerror(L.ESCRATCH)
    rc = lib.ljmd_lj_backward_noalloc(None, None, n, ctypes.byref(b), ctypes.byref(p),
                                      ctypes.byref(nl), d, 0, d, None, None, None)
    assert rc == L.EINVAL


def test_fm_grad_validation(lib):
    """The one-call force-matching gradient checks its arguments before any
    HIP call: full list only, target forces required, workspace size."""
    b, p = cbox(), cparams()
    d = ctypes.c_void_p(0x1000)
    nl = fake_nlist(10, L.HALF)
    rc = lib.ljmd_fm_grad(d, None, 10, ctypes.byref(b), ctypes.byref(p), ctypes.byref(nl), d,
                          None, 0, None, d, None, None, d, 1 << 30, None)
    assert rc == L.ENOTSUP  # half list
    nl = fake_nlist(10)  # global format, 3 x 3 x 3 cells, build strips of 3 cells
    for k in range(3):
        nl.ncell[k] = 3
        nl.tile[k] = 3 if k == 0 else 1
    rc = lib.ljmd_fm_grad(d, None, 10, ctypes.byref(b), ctypes.byref(p), ctypes.byref(nl), None,
                          None, 0, None, d, None, None, d, 1 << 30, None)
    assert rc == L.EINVAL  # no target forces
    rc = lib.ljmd_fm_grad(d, None, 10, ctypes.byref(b), ctypes.byref(p), ctypes.byref(nl), d,
                          None, L.PREC_MIXED, None, d, None, None, d, 16, None)
    assert rc == L.EWORKSPACE  # mixed forward accepted, workspace too small


def test_python_params_roundtrip(lib):
    eps, sig, rc = inputs.binary_tables()
    prm = api.LJParams(eps=eps, sigma=sig, rc=rc, skin=0.3, mass=[1.0, 2.0])
    c = prm.to_c()
    assert c.ntypes == 2 and c.eps[0][1] == 1.5 and c.sigma[1][1] == 0.88 and c.rc[1][0] == 2.0
    assert c.mass[1] == 2.0 and c.skin == 0.3
    assert api.workspace_bytes(500, [7.5] * 3, prm) > 0
    with pytest.raises(L.LjmdError) as e:
        api.workspace_bytes(500, [5.0] * 3, prm)
    assert e.value.code == L.EBOX


def test_thermo_row_count():
    assert api.thermo_rows(0, 100, 10, True) == 11
    assert api.thermo_rows(0, 100, 10, False) == 10
    assert api.thermo_rows(5, 20, 10, False) == 2   # 10, 20
    assert api.thermo_rows(5, 20, 10, True) == 2
    assert api.thermo_rows(10, 0, 10, True) == 1
    assert api.thermo_rows(0, 100, 0, True) == 0


def test_product_path_refuses_without_library(monkeypatch, tmp_path):
    """No fallback: a missing library is an error, not a silent CPU path."""
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="libljmd.so not found"):
        L.load()
    np.testing.assert_equal(1, 1)


def cbatch(sizes, box_len, dev_ptrs=True):
    """A batch struct over host arrays (kept alive on the returned object)."""
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    boxes = np.array([[b, b, b] for b in box_len], dtype=np.float64)
    bt = L.Batch()
    bt.nrep = len(sizes)
    bt.offsets = off.ctypes.data
    bt.boxes = boxes.ctypes.data
    bt.d_offsets = 0x1000 if dev_ptrs else None
    bt.d_boxes = 0x1000 if dev_ptrs else None
    bt._keep = (off, boxes)
    return bt


def test_batch_sizes_and_validation(lib):
    p = cparams()
    b = cbatch([100, 200, 300], [10.0, 12.0, 14.0])
    w = lib.ljmd_batch_workspace_bytes(ctypes.byref(b), ctypes.byref(p), 0)
    a = lib.ljmd_batch_aux_bytes(ctypes.byref(b), ctypes.byref(p))
    assert w > 0 and w % 256 == 0 and a > 0
    # a larger batch needs more scratch
    b2 = cbatch([100, 200, 300, 400], [10.0, 12.0, 14.0, 16.0])
    assert lib.ljmd_batch_workspace_bytes(ctypes.byref(b2), ctypes.byref(p), 0) > w
    # tile targets: 0 (the default 300) or 32 .. 4096; smaller tiles, more of them
    for bad_target in (5, 31, 4097):
        bt = cbatch([100, 200, 300], [10.0, 12.0, 14.0])
        bt.tile_atoms = bad_target
        assert lib.ljmd_batch_workspace_bytes(ctypes.byref(bt), ctypes.byref(p), 0) == 0
    small = cbatch([4000, 4000], [15.0, 15.0])
    small.tile_atoms = 64
    large = cbatch([4000, 4000], [15.0, 15.0])
    large.tile_atoms = 1000
    assert (lib.ljmd_batch_workspace_bytes(ctypes.byref(small), ctypes.byref(p), 0) >
            lib.ljmd_batch_workspace_bytes(ctypes.byref(large), ctypes.byref(p), 0) > 0)
    # a box shorter than twice the neighbor cutoff, non-monotone offsets, no systems
    assert lib.ljmd_batch_workspace_bytes(ctypes.byref(cbatch([10, 10], [10.0, 5.0])),
                                          ctypes.byref(p), 0) == 0
    bad = cbatch([10, 10], [10.0, 10.0])
    bad._keep[0][2] = 5  # offsets 0, 10, 5
    assert lib.ljmd_batch_workspace_bytes(ctypes.byref(bad), ctypes.byref(p), 0) == 0
    empty = cbatch([], [])
    assert lib.ljmd_batch_workspace_bytes(ctypes.byref(empty), ctypes.byref(p), 0) == 0
    # systems whose cell grids together exceed the int32 cell tables
    big = cbatch([10, 10], [3000.0, 3000.0])
    assert lib.ljmd_batch_workspace_bytes(ctypes.byref(big), ctypes.byref(p), 0) == 0
    rc = lib.ljmd_batch_nl_build(ctypes.c_void_p(0x1000), None, ctypes.byref(big),
                                 ctypes.byref(p), ctypes.byref(fake_nlist(20)),
                                 ctypes.c_void_p(0x1000), 1 << 30, None)
    assert rc == L.ENOTSUP
    d = ctypes.c_void_p(0x1000)
    nl = fake_nlist(600)
    rc = lib.ljmd_batch_nl_build(d, None, ctypes.byref(cbatch([10, 10], [10.0, 5.0])),
                                 ctypes.byref(p), ctypes.byref(nl), d, 1 << 30, None)
    assert rc == L.EBOX
    rc = lib.ljmd_batch_nl_build(d, None, ctypes.byref(b), ctypes.byref(p), ctypes.byref(nl), d,
                                 16, None)
    assert rc == L.EWORKSPACE
    nl_h = fake_nlist(600, L.HALF)
    rc = lib.ljmd_batch_nl_build(d, None, ctypes.byref(b), ctypes.byref(p), ctypes.byref(nl_h),
                                 d, 1 << 30, None)
    assert rc == L.ENOTSUP
    nodev = cbatch([100, 200, 300], [10.0, 12.0, 14.0], dev_ptrs=False)
    rc = lib.ljmd_batch_nl_build(d, None, ctypes.byref(nodev), ctypes.byref(p), ctypes.byref(nl),
                                 d, 1 << 30, None)
    assert rc == L.EINVAL
    # forces on a list that was not built for this batch
    nl.format = L.FMT_GLOBAL
    rc = lib.ljmd_batch_lj_forces(d, None, ctypes.byref(b), ctypes.byref(p), ctypes.byref(nl), 0,
                                  d, None, d, 1 << 30, None)
    assert rc == L.EINVAL
    # tuning table: invalid variants are rejected, clearing always works
    t = L.BatchTuning()
    t.lanes_per_atom, t.block, t.persistent = 3, 256, 0
    assert lib.ljmd_batch_set_tuning(ctypes.byref(b), ctypes.byref(p), 0, ctypes.byref(t)) == \
        L.EINVAL
    t.lanes_per_atom = 2
    assert lib.ljmd_batch_set_tuning(ctypes.byref(b), ctypes.byref(p), 0, ctypes.byref(t)) == L.OK
    assert lib.ljmd_batch_set_tuning(ctypes.byref(b), ctypes.byref(p), 0, None) == L.OK


def test_gather_lanes_setting(lib):
    """ljmd_set_gather_lanes accepts 0 (automatic, the default), 1, 2, 4 and
    8, and rejects anything else without changing the setting."""
    before = lib.ljmd_get_gather_lanes()
    try:
        for lanes in (1, 2, 4, 8, 0):
            assert lib.ljmd_set_gather_lanes(lanes) == L.OK
            assert lib.ljmd_get_gather_lanes() == lanes
        assert lib.ljmd_set_gather_lanes(2) == L.OK
        for bad in (3, -1, 16, 64):
            assert lib.ljmd_set_gather_lanes(bad) == L.EINVAL
            assert lib.ljmd_get_gather_lanes() == 2
    finally:
        lib.ljmd_set_gather_lanes(before)


def test_pair_table_gradients():
    """pair_table: the symmetric table from the unique type-pair values; the
    gradient of an off-diagonal value sums its two mirrored entries."""
    import torch
    from paper_2508_13523_amd.autograd import pair_table

    u = torch.tensor([1.0, 2.0, 3.0, 4.0, 5.0, 6.0], dtype=torch.float64, requires_grad=True)
    t = pair_table(u, 3)
    assert torch.equal(t, t.T)
    assert t[0, 0] == 1.0 and t[0, 2] == 3.0 and t[1, 2] == 5.0 and t[2, 2] == 6.0
    w = torch.arange(9, dtype=torch.float64).reshape(3, 3)
    (t * w).sum().backward()
    expect = [w[0, 0], w[0, 1] + w[1, 0], w[0, 2] + w[2, 0], w[1, 1], w[1, 2] + w[2, 1], w[2, 2]]
    assert torch.equal(u.grad, torch.stack(expect))
    with pytest.raises(ValueError):
        pair_table(u[:5], 3)
