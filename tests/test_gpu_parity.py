"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Bars: neighbor lists bit-exact as sets (FP64 distance tests with the same
operation order on both sides); FP64 forces within 1e-12 normwise
(max |dF| / max |F_ref|), energy and virial within 1e-12 relative; mixed
precision within the per-atom rounding bound of its FP32 pair terms
(tests/mixed_bound.py: |dF_i| <= 25 u sum_j |f_ij|, u = 2^-24) and within
2e-6 normwise; trajectories within 1e-9 over 100 steps.
"""
import math

import numpy as np
import pytest
import torch

from paper_2508_13523_amd import _lib as L
from paper_2508_13523_amd import api, inputs

from mixed_bound import check_mixed

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda"


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def types_of(s):
    return dev(s.types, torch.int32) if s.ntypes > 1 else None


def params_of(s):
    return api.LJParams.from_system(s)


def rel_err(a, b):
    scale = np.abs(b).max()
    return np.abs(a - b).max() / (scale if scale > 0 else 1.0)


def assert_rows_equal(gpu_csr, ref_csr):
    c, o, i = gpu_csr[:3]
    rc, ro, ri = ref_csr
    assert np.array_equal(c, rc), f"row counts differ at {np.nonzero(c != rc)[0][:10]}"
    assert np.array_equal(i, ri)


def pair_keys(csr, n):
    """The list's pairs as sorted keys min(i,j) * n + max(i,j)."""
    c, _, i = csr[:3]
    rows = np.repeat(np.arange(len(c), dtype=np.int64), c)
    j = np.asarray(i, dtype=np.int64)
    return np.sort(np.minimum(rows, j) * n + np.maximum(rows, j))


def assert_half_equal(gpu_csr, ref_csr):
    """Half lists as sets of unordered pairs (the owner row of a pair differs:
    the oracle lists it in row min(i,j), the tiled GPU list in the row of the
    atom that comes first in its tile's stencil order), each pair once."""
    n = len(ref_csr[0])
    got, want = pair_keys(gpu_csr, n), pair_keys(ref_csr, n)
    assert np.unique(got).size == got.size, "a pair is listed twice"
    assert np.array_equal(got, want)


def assert_list_equal(gpu_csr, ref_csr, half):
    if half:
        assert_half_equal(gpu_csr, ref_csr)
    else:
        assert_rows_equal(gpu_csr, ref_csr)


def check_ev(ev, ev_ref, tol=1e-12):
    scale = np.abs(ev_ref).max()
    assert np.abs(ev - ev_ref).max() <= tol * scale, (ev, ev_ref)


def check_codes(x_wrapped, box, csr):
    """The image code of every entry is the branch taken by the minimum image."""
    c, o, idx, codes = csr
    rows = np.repeat(np.arange(len(c)), c)
    d = x_wrapped[rows] - x_wrapped[idx]
    expect = np.zeros(len(idx), dtype=np.int64)
    for k in range(3):
        h = 0.5 * box[k]
        expect |= np.where(d[:, k] > h, 1, np.where(d[:, k] < -h, 2, 0)) << (2 * k)
    assert np.array_equal(codes, expect)


# ---------------------------------------------------------------- systems


@pytest.fixture(scope="module")
def c1():
    return inputs.fcc_liquid(10)  # 4,000 atoms, 5 cells per dimension


@pytest.fixture(scope="module")
def binary2k():
    return inputs.binary_liquid(2000, seed=17)


@pytest.fixture(scope="module")
def binary500():
    return inputs.binary_liquid(500, seed=19)  # L = 7.47: 2 cells per dimension


@pytest.fixture(scope="module")
def ortho():
    return inputs.fcc_liquid((9, 6, 12))  # 2,592 atoms, 15.1 x 10.1 x 20.2: 5 x 3 x 7 cells


@pytest.fixture(scope="module")
def ortho_thin():
    return inputs.fcc_liquid((12, 4, 9))  # 1,728 atoms, 20.2 x 6.7 x 15.1: 7 x 2 x 5 cells


# ---------------------------------------------------------------- neighbor lists


FMTS = ["tiled", "global"]


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("mode", ["full", "half"])
def test_nl_c1(oracle, c1, mode, fmt):
    s = c1
    x = dev(s.x)
    nl = api.build_list(x, None, s.box, params_of(s), mode=mode, global_format=fmt == "global")
    assert nl.format == fmt
    xw = oracle.wrap(s.x, s.box)
    assert np.array_equal(x.cpu().numpy(), xw)
    csr = nl.to_csr()
    assert_list_equal(csr, oracle.nl_brute(s.x, None, s.box, s.rc, s.skin, mode == "half"),
                      mode == "half")
    check_codes(xw, s.box, csr)
    st = api.get_status(nl)
    assert st[L.ST_OVERFLOW] == 0 and st[L.ST_NEED] == csr[0].max()


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("mode", ["full", "half"])
@pytest.mark.parametrize("case", ["binary500", "binary2k", "dense1.1", "ragged", "outside"])
def test_nl_edge_cases(oracle, case, mode, fmt, binary500, binary2k):
    if case == "binary500":
        s = binary500
    elif case == "binary2k":
        s = binary2k
    elif case == "dense1.1":
        s = inputs.fcc_liquid(4, rho=1.1)  # L = 6.15: 2 cells per dimension
    elif case == "ragged":
        s = inputs.fcc_liquid(7)
        keep = np.sort(np.random.default_rng(3).choice(s.n, s.n - 37, replace=False))
        s.x, s.v, s.types = s.x[keep], s.v[keep], s.types[keep]
    else:  # coordinates on and just outside the box faces, wrapped by the build
        s = inputs.fcc_liquid(6)
        s.x = s.x.copy()
        s.x[:40] -= 0.07
        s.x[40:80, 0] = 0.0
        s.x[80:120, 1] = s.box[1] + 0.03
        s.x[120] = [-1e-17, 0.0, s.box[2] - 1e-15]
    x = dev(s.x)
    nl = api.build_list(x, types_of(s), s.box, params_of(s), mode=mode,
                        global_format=fmt == "global")
    # boxes with fewer than 3 cells per dimension always use the global format
    small = case in ("binary500", "dense1.1")
    assert nl.format == ("global" if small else fmt)
    xw = oracle.wrap(s.x, s.box)
    assert np.array_equal(x.cpu().numpy(), xw)
    csr = nl.to_csr()
    assert_list_equal(csr, oracle.nl_brute(s.x, s.types, s.box, s.rc, s.skin, mode == "half"),
                      mode == "half")
    check_codes(xw, s.box, csr)
    # forces over this list as well
    f, ev = api.lj_forces(x, types_of(s), s.box, params_of(s), nl, ev=True)
    f_ref, ev_ref = oracle.forces_brute(xw, s.types, s.box, s.eps, s.sigma, s.rc)
    assert rel_err(f.cpu().numpy(), f_ref) < 1e-12
    check_ev(ev.cpu().numpy(), ev_ref)


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("mode", ["full", "half"])
@pytest.mark.parametrize("case", ["ortho", "ortho_thin"])
def test_orthorhombic_lists_and_forces(oracle, case, mode, fmt, ortho, ortho_thin):
    """A different length and cell count along each axis (the tiles, the x
    windows and the minimum image per axis): lists bit-exact as sets against
    brute force, FP64 forces within 1e-12 and energy/virial within 1e-12, the
    mixed forces within their rounding bound.  With 2 cells along y the thin
    box takes the global format."""
    s = ortho if case == "ortho" else ortho_thin
    x = dev(s.x)
    prm = params_of(s)
    nl = api.build_list(x, None, s.box, prm, mode=mode, global_format=fmt == "global")
    assert nl.format == ("global" if case == "ortho_thin" else fmt)
    xw = oracle.wrap(s.x, s.box)
    csr = nl.to_csr()
    assert_list_equal(csr, oracle.nl_brute(s.x, s.types, s.box, s.rc, s.skin, mode == "half"),
                      mode == "half")
    check_codes(xw, s.box, csr)
    f, ev = api.lj_forces(x, None, s.box, prm, nl, ev=True)
    f_ref, ev_ref = oracle.forces_brute(xw, s.types, s.box, s.eps, s.sigma, s.rc)
    assert rel_err(f.cpu().numpy(), f_ref) < 1e-12
    check_ev(ev.cpu().numpy(), ev_ref)
    fm, evm = api.lj_forces(x, None, s.box, prm, nl, mixed=True, ev=True)
    check_mixed(fm.cpu().numpy(), evm.cpu().numpy(), f_ref, ev_ref, xw, s.types, s.box, s.eps,
                s.sigma, s.rc, oracle.nl_brute(s.x, s.types, s.box, s.rc, 0.0))


def seeded_grid_system(seed):
    """Seeded variety: density 0.6, 0.8442, 1.1 or 1.2, 7-18 grid sites per
    axis (boxes of 2-7 cells per axis, so some take the global format), one
    type or the binary mixture, sites jittered by N(0, 0.05^2)."""
    rng = np.random.default_rng(1000 + seed)
    rho = [0.6, 0.8442, 1.1, 1.2][seed % 4]
    return inputs.grid_system(rng.integers(7, 19, size=3), rho, seed, binary=bool(seed % 2),
                              jitter_std=0.05)


@pytest.mark.parametrize("seed", range(8))
def test_seeded_systems(oracle, seed):
    """Lists (full and half, tiled and global) bit-exact as sets against
    brute force, FP64 forces, energy and virial within 1e-12, mixed forces
    within their rounding bound, the adjoint's gradients within 1e-11, and
    40 MD steps (dt = 0.002: the dense grid
    starts are far from equilibrium) with atom sorting against the oracle's
    run, on seeded systems of varied density, shape and types."""
    s = seeded_grid_system(seed)
    x = dev(s.x)
    t = types_of(s)
    prm = params_of(s)
    xw = oracle.wrap(s.x, s.box)
    f_ref, ev_ref = oracle.forces_brute(xw, s.types, s.box, s.eps, s.sigma, s.rc)
    g = np.random.default_rng(seed + 5).normal(size=(s.n, 3))
    bx_ref, be_ref, bs_ref = oracle.backward_brute(xw, s.types, s.box, s.eps, s.sigma, s.rc, g)
    small = bool(np.any(np.floor(s.box / (float(np.max(s.rc)) + s.skin) / (1 + 1e-12)) < 3))
    for mode in ("full", "half"):
        ref = oracle.nl_brute(s.x, s.types, s.box, s.rc, s.skin, mode == "half")
        for fmt in FMTS:
            nl = api.build_list(x, t, s.box, prm, mode=mode, global_format=fmt == "global")
            assert nl.format == ("global" if small else fmt)
            assert_list_equal(nl.to_csr(), ref, mode == "half")
            f, ev = api.lj_forces(x, t, s.box, prm, nl, ev=True)
            assert rel_err(f.cpu().numpy(), f_ref) < 1e-12, (mode, fmt)
            check_ev(ev.cpu().numpy(), ev_ref)
            if mode == "full":
                fm, evm = api.lj_forces(x, t, s.box, prm, nl, mixed=True, ev=True)
                check_mixed(fm.cpu().numpy(), evm.cpu().numpy(), f_ref, ev_ref, xw, s.types,
                            s.box, s.eps, s.sigma, s.rc,
                            oracle.nl_brute(s.x, s.types, s.box, s.rc, 0.0))
                # the adjoint: gradients to positions and to the eps / sigma tables
                gx, geps, gsig = api.lj_backward(x, t, s.box, prm, nl, dev(g))
                assert rel_err(gx.cpu().numpy(), bx_ref) < 1e-11, fmt
                assert rel_err(geps.cpu().numpy(), be_ref) < 1e-11, fmt
                assert rel_err(gsig.cpu().numpy(), bs_ref) < 1e-11, fmt
    v = dev(s.v)
    f = torch.zeros_like(x)
    ids = torch.arange(s.n, dtype=torch.int32, device=DEV)
    nl = api.NeighborList(s.n, api.default_capacity(prm, s.box, s.n), s.box, prm)
    api.md_step(x, v, f, t, s.box, prm, nl, 0.002, 40, rebuild_every=10, setup=True, sort=True,
                ids=ids, sync_check=True)
    xr, vr, fr, _ = oracle.md(s.x, s.v, s.types, s.box, s.eps, s.sigma, s.rc, s.mass, 0.002, 40,
                              rebuild_every=10, skin=s.skin)
    idn = ids.cpu().numpy()
    assert np.abs(x.cpu().numpy() - xr[idn]).max() < 1e-9
    assert np.abs(v.cpu().numpy() - vr[idn]).max() < 1e-8
    assert rel_err(f.cpu().numpy(), fr[idn]) < 1e-9


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("mode", ["full", "half"])
def test_nl_export_indices(c1, mode, fmt):
    """The plain index layout (entry k of row i at k * n + i, user indices)
    holds the same rows as the interleaved export with image codes."""
    s = c1
    x = dev(s.x)
    nl = api.build_list(x, None, s.box, params_of(s), mode=mode, global_format=fmt == "global")
    idx, counts = nl.export_indices()
    idx, counts = idx.cpu().numpy(), counts.cpu().numpy()
    c, o, i = nl.to_csr()[:3]
    assert np.array_equal(counts, c)
    k = np.arange(nl.cap)[:, None]
    assert np.all(idx[k >= counts[None, :]] == -1)  # untouched beyond each row
    for a in range(s.n):
        assert np.array_equal(np.sort(idx[: counts[a], a]), i[o[a]:o[a + 1]]), a


@pytest.mark.parametrize("mode", ["full", "half"])
def test_nl_large_cells_chunked(oracle, mode):
    """Cells of 7.5 at density 1 (about 420 atoms per cell): more home atoms per
    workgroup than threads and more stencil-row atoms than one LDS chunk (the
    build and the scatter then stage the stencil in chunks)."""
    x0, box = inputs.random_sites(27000, 1.0, seed=23)
    eps, sig, rc = inputs.single_type_tables(rc=7.0)
    prm = api.LJParams(eps=eps, sigma=sig, rc=rc, skin=0.3)
    x = dev(x0)
    nl = api.build_list(x, None, box, prm, mode=mode)
    assert nl.format == "tiled"
    ref = oracle.nl_cells(x0, None, box, rc, 0.3, mode == "half")
    assert_list_equal(nl.to_csr(), ref, mode == "half")
    f, ev = api.lj_forces(x, None, box, prm, nl, ev=True)
    f_ref, ev_ref = oracle.forces_cells(oracle.wrap(x0, box), None, box, eps, sig, rc)
    assert rel_err(f.cpu().numpy(), f_ref) < 1e-12


def test_nl_tiny_and_empty(oracle):
    prm = api.LJParams(*inputs.single_type_tables(), skin=0.3)
    box = np.full(3, 6.0)
    # one atom: empty row, zero force
    x = dev([[1.0, 2.0, 3.0]])
    nl = api.build_list(x, None, box, prm)
    assert nl.numneigh.cpu().numpy()[0] == 0
    f, ev = api.lj_forces(x, None, box, prm, nl, ev=True)
    assert np.all(f.cpu().numpy() == 0) and np.all(ev.cpu().numpy() == 0)
    # no atoms at all
    x0 = torch.zeros((0, 3), dtype=torch.float64, device=DEV)
    nl0 = api.NeighborList(0, 4, box, prm)
    api.nl_build(x0, None, box, prm, nl0)
    f0, ev0 = api.lj_forces(x0, None, box, prm, nl0, ev=True)
    assert f0.shape == (0, 3) and np.all(ev0.cpu().numpy() == 0)
    # two atoms through every face pair
    for k in range(3):
        p = np.full((2, 3), 3.0)
        p[0, k], p[1, k] = 0.2, 5.7
        x = dev(p)
        nl = api.build_list(x, None, box, prm)
        c, o, idx, codes = nl.to_csr()
        assert list(c) == [1, 1] and list(idx) == [1, 0]
        assert codes[0] == 2 << (2 * k) and codes[1] == 1 << (2 * k)


def test_nl_overflow_reports_need(oracle, c1):
    s = c1
    x = dev(s.x)
    nl = api.NeighborList(s.n, 40, s.box, params_of(s))
    api.nl_build(x, None, s.box, params_of(s), nl)
    st = api.get_status(nl)
    ref_counts = oracle.nl_brute(s.x, None, s.box, s.rc, s.skin)[0]
    assert st[L.ST_OVERFLOW] == 1 and st[L.ST_NEED] == ref_counts.max()
    assert np.array_equal(nl.numneigh.cpu().numpy(), np.minimum(ref_counts, 40))
    # the regrowing builder ends with a complete list
    nl2 = api.build_list(x, None, s.box, params_of(s), cap=40)
    assert nl2.cap >= ref_counts.max()
    assert api.get_status(nl2)[L.ST_OVERFLOW] == 0


# ---------------------------------------------------------------- forces


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("mode", ["full", "half"])
@pytest.mark.parametrize("case", ["c1", "binary2k", "binary500"])
def test_forces_fp64(oracle, case, mode, fmt, c1, binary2k, binary500):
    s = {"c1": c1, "binary2k": binary2k, "binary500": binary500}[case]
    x = dev(s.x)
    prm = params_of(s)
    nl = api.build_list(x, types_of(s), s.box, prm, mode=mode, global_format=fmt == "global")
    f, ev = api.lj_forces(x, types_of(s), s.box, prm, nl, ev=True)
    xw = oracle.wrap(s.x, s.box)
    f_ref, ev_ref = oracle.forces_brute(xw, s.types, s.box, s.eps, s.sigma, s.rc)
    assert rel_err(f.cpu().numpy(), f_ref) < 1e-12
    check_ev(ev.cpu().numpy(), ev_ref)
    # forces without energy/virial are the same numbers
    f2, _ = api.lj_forces(x, types_of(s), s.box, prm, nl, ev=False)
    assert rel_err(f2.cpu().numpy(), f_ref) < 1e-12


@pytest.fixture
def gather_lanes():
    """Restores the process-wide gather lanes setting after the test."""
    before = api.get_gather_lanes()
    yield
    api.set_gather_lanes(before)


@pytest.mark.parametrize("lanes", [1, 2, 4, 8])
@pytest.mark.parametrize("case", ["c1", "binary2k", "large_cells"])
def test_gather_lanes_per_atom(oracle, gather_lanes, case, lanes, c1, binary2k):
    """1, 2, 4 or 8 lanes per atom in the tiled gather: FP64 forces, energy and
    virial to the 1e-12 bar, mixed to its rounding bound.  large_cells (about 420
    atoms per cell) has stencils too large for LDS, which takes the chunked
    path where each lane walks every lanes-th word of its row."""
    if case == "large_cells":
        x0, box = inputs.random_sites(27000, 1.0, seed=23)
        eps, sig, rc = inputs.single_type_tables(rc=7.0)
        prm = api.LJParams(eps=eps, sigma=sig, rc=rc, skin=0.3)
        types = None
        f_ref, ev_ref = oracle.forces_cells(oracle.wrap(x0, box), None, box, eps, sig, rc)
        csr = oracle.nl_cells(x0, None, box, rc, 0.0)
    else:
        s = {"c1": c1, "binary2k": binary2k}[case]
        x0, box, prm, types = s.x, s.box, params_of(s), s.types if s.ntypes > 1 else None
        eps, sig, rc = s.eps, s.sigma, s.rc
        f_ref, ev_ref = oracle.forces_brute(oracle.wrap(s.x, s.box), s.types, s.box, s.eps,
                                            s.sigma, s.rc)
        csr = oracle.nl_brute(s.x, s.types, s.box, s.rc, 0.0)
    x = dev(x0)
    t = dev(types, torch.int32) if types is not None else None
    nl = api.build_list(x, t, box, prm)
    assert nl.format == "tiled"
    api.set_gather_lanes(lanes)
    assert api.get_gather_lanes() == lanes
    f, ev = api.lj_forces(x, t, box, prm, nl, ev=True)
    assert rel_err(f.cpu().numpy(), f_ref) < 1e-12
    check_ev(ev.cpu().numpy(), ev_ref)
    f2, _ = api.lj_forces(x, t, box, prm, nl)
    assert torch.equal(f, f2)
    fm, evm = api.lj_forces(x, t, box, prm, nl, mixed=True, ev=True)
    check_mixed(fm.cpu().numpy(), evm.cpu().numpy(), f_ref, ev_ref, oracle.wrap(x0, box),
                types, box, eps, sig, rc, csr)


def test_gather_is_bitwise_deterministic(c1):
    s = c1
    x = dev(s.x)
    nl = api.build_list(x, None, s.box, params_of(s))
    a, ea = api.lj_forces(x, None, s.box, params_of(s), nl, ev=True)
    b, eb = api.lj_forces(x, None, s.box, params_of(s), nl, ev=True)
    assert torch.equal(a, b) and torch.equal(ea, eb)


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("mode", ["full", "half"])
@pytest.mark.parametrize("case", ["c1", "binary2k"])
def test_forces_mixed(oracle, case, mode, fmt, c1, binary2k):
    """FP32 pair terms, FP64 everything else: every atom's force within the
    rounding bound of its FP32 pair terms (25 u per pair magnitude, summed
    over the atom's partners), 2e-6 of max |F| overall, energy and virial
    within the same per-pair bound summed over the system.  The measured
    largest |dF_i| / sum_j |f_ij| is printed."""
    s = {"c1": c1, "binary2k": binary2k}[case]
    x = dev(s.x)
    prm = params_of(s)
    nl = api.build_list(x, types_of(s), s.box, prm, mode=mode, global_format=fmt == "global")
    f, ev = api.lj_forces(x, types_of(s), s.box, prm, nl, mixed=True, ev=True)
    xw = oracle.wrap(s.x, s.box)
    f_ref, ev_ref = oracle.forces_brute(xw, s.types, s.box, s.eps, s.sigma, s.rc)
    csr = oracle.nl_brute(s.x, s.types, s.box, s.rc, 0.0)
    worst = check_mixed(f.cpu().numpy(), ev.cpu().numpy(), f_ref, ev_ref, xw, s.types, s.box,
                        s.eps, s.sigma, s.rc, csr)
    print(f"mixed {case} {mode} {fmt}: max |dF_i|/S_i = {worst:.3e} (bound {25 * 2**-24:.3e}), "
          f"normwise {rel_err(f.cpu().numpy(), f_ref):.3e}")


# ---------------------------------------------------------------- integrator


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("mode", ["full", "half"])
def test_md_c1_100_steps(oracle, c1, mode, fmt):
    """4,000 atoms, 100 velocity-Verlet steps, rebuild every 20."""
    s = c1
    x, v = dev(s.x), dev(s.v)
    f = torch.zeros_like(x)
    prm = params_of(s)
    nl = api.NeighborList(s.n, api.default_capacity(prm, s.box, s.n), s.box, prm, mode=mode,
                          global_format=fmt == "global")
    th = api.md_step(x, v, f, None, s.box, prm, nl, s.dt, 100, rebuild_every=20,
                     thermo_every=10, setup=True, sync_check=True)
    xr, vr, fr, thr = oracle.md(s.x, s.v, None, s.box, s.eps, s.sigma, s.rc, s.mass, s.dt, 100,
                                rebuild_every=20, thermo_every=10, skin=s.skin)
    assert np.abs(x.cpu().numpy() - xr).max() < 1e-9
    assert np.abs(v.cpu().numpy() - vr).max() < 1e-8
    assert rel_err(f.cpu().numpy(), fr) < 1e-9
    th = th.cpu().numpy()
    assert th.shape == thr.shape == (11, 9)
    assert np.array_equal(th[:, 0], thr[:, 0])
    assert np.allclose(th[:, 1:], thr[:, 1:], rtol=1e-9, atol=1e-9 * np.abs(thr[:, 1:]).max())
    st = api.get_status(nl)
    # T = 1.44 with skin 0.3 and a rebuild every 20 steps: some atoms do move
    # more than skin/2 between builds, which the status word reports
    assert st[L.ST_OVERFLOW] == 0 and st[L.ST_NONFINITE] == 0


def test_md_binary_small_box(oracle, binary500):
    s = binary500
    x, v = dev(s.x), dev(s.v)
    f = torch.zeros_like(x)
    prm = params_of(s)
    t = types_of(s)
    nl = api.NeighborList(s.n, api.default_capacity(prm, s.box, s.n), s.box, prm)
    th = api.md_step(x, v, f, t, s.box, prm, nl, s.dt, 60, rebuild_every=20, thermo_every=20,
                     setup=True)
    xr, vr, fr, thr = oracle.md(s.x, s.v, s.types, s.box, s.eps, s.sigma, s.rc, s.mass, s.dt, 60,
                                rebuild_every=20, thermo_every=20, skin=s.skin)
    assert np.abs(x.cpu().numpy() - xr).max() < 1e-9
    assert np.allclose(th.cpu().numpy(), thr, rtol=1e-9, atol=1e-9 * np.abs(thr).max())


@pytest.mark.parametrize("case", ["ortho", "ortho_thin"])
def test_md_orthorhombic(oracle, case, ortho, ortho_thin):
    """100 steps, rebuild every 20, in boxes with a different length per axis
    (tiled with the fused update, and global), against the oracle's run."""
    s = ortho if case == "ortho" else ortho_thin
    x, v = dev(s.x), dev(s.v)
    f = torch.zeros_like(x)
    prm = params_of(s)
    nl = api.NeighborList(s.n, api.default_capacity(prm, s.box, s.n), s.box, prm)
    th = api.md_step(x, v, f, None, s.box, prm, nl, s.dt, 100, rebuild_every=20,
                     thermo_every=20, setup=True, sync_check=True)
    xr, vr, fr, thr = oracle.md(s.x, s.v, None, s.box, s.eps, s.sigma, s.rc, s.mass, s.dt, 100,
                                rebuild_every=20, thermo_every=20, skin=s.skin)
    assert nl.format == ("global" if case == "ortho_thin" else "tiled")
    assert np.abs(x.cpu().numpy() - xr).max() < 1e-9
    assert np.abs(v.cpu().numpy() - vr).max() < 1e-8
    assert rel_err(f.cpu().numpy(), fr) < 1e-9
    assert np.allclose(th.cpu().numpy(), thr, rtol=1e-9, atol=1e-9 * np.abs(thr).max())


@pytest.mark.parametrize("case", ["c1", "binary500", "binary2k", "ortho"])
def test_md_sorted_atoms(oracle, case, c1, binary500, binary2k, ortho):
    """With atom sorting the trajectory is the oracle's, permuted: ids say which
    oracle atom each slot holds, types travel with their atoms, and after the
    run atoms are in cell order and the list matches the oracle's."""
    s = {"c1": c1, "binary500": binary500, "binary2k": binary2k, "ortho": ortho}[case]
    prm = params_of(s)
    x, v = dev(s.x), dev(s.v)
    f = torch.zeros_like(x)
    t = types_of(s)
    ids = torch.arange(s.n, dtype=torch.int32, device=DEV)
    nl = api.NeighborList(s.n, api.default_capacity(prm, s.box, s.n), s.box, prm)
    th = api.md_step(x, v, f, t, s.box, prm, nl, s.dt, 100, rebuild_every=20, thermo_every=20,
                     setup=True, sort=True, ids=ids)
    xr, vr, fr, thr = oracle.md(s.x, s.v, s.types, s.box, s.eps, s.sigma, s.rc, s.mass, s.dt,
                                100, rebuild_every=20, thermo_every=20, skin=s.skin)
    idn = ids.cpu().numpy()
    assert np.array_equal(np.sort(idn), np.arange(s.n))
    assert not np.array_equal(idn, np.arange(s.n))
    assert np.abs(x.cpu().numpy() - xr[idn]).max() < 1e-9
    assert np.abs(v.cpu().numpy() - vr[idn]).max() < 1e-8
    assert rel_err(f.cpu().numpy(), fr[idn]) < 1e-9
    assert np.allclose(th.cpu().numpy(), thr, rtol=1e-9, atol=1e-9 * np.abs(thr).max())
    if t is not None:
        assert np.array_equal(t.cpu().numpy(), s.types[idn])
    # the last build (step 100) sorted the atoms: cell index non-decreasing
    xh = x.cpu().numpy()
    nc = np.floor(s.box / (float(np.max(s.rc)) + s.skin) / (1 + 1e-12)).astype(int)
    cc = np.minimum((xh * nc / s.box).astype(int), nc - 1)
    cell = (cc[:, 2] * nc[1] + cc[:, 1]) * nc[0] + cc[:, 0]
    assert np.all(np.diff(cell) >= 0)
    ts = t.cpu().numpy() if t is not None else None
    assert_rows_equal(nl.to_csr(), oracle.nl_brute(xh, ts, s.box, s.rc, s.skin))


@pytest.mark.parametrize("sort", [False, True])
def test_md_graph_replays_equal_eager(c1, sort):
    """A HIP graph captured around the single-system MD step (fused kick,
    rebuilds inside, atoms re-sorted at each rebuild when sort) reproduces the
    eager run on every replay, with eager work and synchronizations between
    the replays."""
    s = c1
    prm = params_of(s)
    x0, v0 = dev(s.x), dev(s.v)
    f0 = torch.zeros_like(x0)
    nl = api.NeighborList(s.n, api.default_capacity(prm, s.box, s.n), s.box, prm)
    ws = api.workspace(s.n, s.box, prm)
    api.md_step(x0, v0, f0, None, s.box, prm, nl, s.dt, 5, setup=True, ws=ws, sort=sort)
    bufs = (x0, v0, f0, nl.neigh, nl.numneigh, nl.aux, nl.xref)
    state0 = [a.clone() for a in bufs]
    thermo = torch.zeros((4, 9), dtype=torch.float64, device=DEV)

    def restore():
        for dst, src in zip(bufs, state0):
            dst.copy_(src)

    def run():
        api.md_step(x0, v0, f0, None, s.box, prm, nl, s.dt, 40, step0=5, rebuild_every=20,
                    thermo_every=10, ws=ws, thermo=thermo, sort=sort)

    restore()
    run()
    torch.cuda.synchronize()
    ref = [a.clone() for a in (x0, v0, f0, thermo)]
    restore()
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            run()
    torch.cuda.current_stream().wait_stream(st)
    torch.cuda.synchronize()
    for rep in range(3):
        restore()
        thermo.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for got, want in zip((x0, v0, f0, thermo), ref):
            assert torch.equal(got, want), rep
        api.lj_forces(x0, None, s.box, prm, nl, ws=ws)  # eager work between replays
        torch.cuda.synchronize()


def test_md_split_calls_equal_one_call(c1):
    """Two calls of 50 steps (the second without set-up) equal one call of 100."""
    s = c1
    prm = params_of(s)
    cap = api.default_capacity(prm, s.box, s.n)
    x1, v1 = dev(s.x), dev(s.v)
    f1 = torch.zeros_like(x1)
    nl1 = api.NeighborList(s.n, cap, s.box, prm)
    api.md_step(x1, v1, f1, None, s.box, prm, nl1, s.dt, 100, setup=True)
    x2, v2 = dev(s.x), dev(s.v)
    f2 = torch.zeros_like(x2)
    nl2 = api.NeighborList(s.n, cap, s.box, prm)
    api.md_step(x2, v2, f2, None, s.box, prm, nl2, s.dt, 50, setup=True)
    api.md_step(x2, v2, f2, None, s.box, prm, nl2, s.dt, 50, step0=50)
    assert torch.equal(x1, x2) and torch.equal(v1, v2) and torch.equal(f1, f2)


@pytest.mark.parametrize("split", [(37, 63), (1, 99), (64, 36)])
def test_md_split_calls_any_parity(c1, split):
    """Calls whose step counts are odd or even (the fused update's position
    buffers then start in x or in the workspace copy) equal one call of 100
    steps bit for bit."""
    s = c1
    prm = params_of(s)
    cap = api.default_capacity(prm, s.box, s.n)
    x1, v1 = dev(s.x), dev(s.v)
    f1 = torch.zeros_like(x1)
    nl1 = api.NeighborList(s.n, cap, s.box, prm)
    api.md_step(x1, v1, f1, None, s.box, prm, nl1, s.dt, 100, setup=True, sort=True)
    x2, v2 = dev(s.x), dev(s.v)
    f2 = torch.zeros_like(x2)
    nl2 = api.NeighborList(s.n, cap, s.box, prm)
    a, b = split
    api.md_step(x2, v2, f2, None, s.box, prm, nl2, s.dt, a, setup=True, sort=True)
    api.md_step(x2, v2, f2, None, s.box, prm, nl2, s.dt, b, step0=a, sort=True)
    assert torch.equal(x1, x2) and torch.equal(v1, v2) and torch.equal(f1, f2)


@pytest.mark.parametrize("case", ["c1", "binary2k"])
@pytest.mark.parametrize("sort", [False, True])
def test_md_fused_kick_equals_separate(case, sort, c1, binary2k):
    """The gather's fused velocity-Verlet update runs the same fmas as the
    separate kick kernels: positions, velocities and forces are bit-identical
    over 45 steps (two rebuilds, odd and even step counts, split calls);
    thermo rows differ only in the summation order of the kinetic energy."""
    s = {"c1": c1, "binary2k": binary2k}[case]
    prm = params_of(s)
    cap = api.default_capacity(prm, s.box, s.n)
    runs = []
    for separate in (False, True):
        x, v = dev(s.x), dev(s.v)
        f = torch.zeros_like(x)
        t = types_of(s)
        ids = torch.arange(s.n, dtype=torch.int32, device=DEV)
        nl = api.NeighborList(s.n, cap, s.box, prm)
        th1 = api.md_step(x, v, f, t, s.box, prm, nl, s.dt, 25, thermo_every=5, setup=True,
                          sort=sort, ids=ids, separate_kick=separate)
        assert nl.format == "tiled"
        th2 = api.md_step(x, v, f, t, s.box, prm, nl, s.dt, 20, step0=25, thermo_every=5,
                          sort=sort, ids=ids, separate_kick=separate)
        runs.append((x, v, f, ids, torch.cat([th1, th2]), api.get_status(nl)))
    (xa, va, fa, ia, tha, sta), (xb, vb, fb, ib, thb, stb) = runs
    assert torch.equal(xa, xb) and torch.equal(va, vb) and torch.equal(fa, fb)
    assert torch.equal(ia, ib) and np.array_equal(sta, stb)
    tha, thb = tha.cpu().numpy(), thb.cpu().numpy()
    assert np.array_equal(tha[:, [0, 1, 3, 4, 5, 6, 7, 8]], thb[:, [0, 1, 3, 4, 5, 6, 7, 8]])
    assert np.allclose(tha[:, 2], thb[:, 2], rtol=1e-13, atol=0)


def test_md_flags_unsafe_rebuild_interval(c1):
    s = c1
    prm = params_of(s)
    x, v = dev(s.x), dev(s.v)
    f = torch.zeros_like(x)
    nl = api.NeighborList(s.n, api.default_capacity(prm, s.box, s.n), s.box, prm)
    api.md_step(x, v, f, None, s.box, prm, nl, 0.005, 40, rebuild_every=4, setup=True)
    assert api.get_status(nl)[L.ST_DANGEROUS] == 0
    api.md_step(x, v, f, None, s.box, prm, nl, 0.012, 40, rebuild_every=20, setup=True)
    assert api.get_status(nl)[L.ST_DANGEROUS] == 1


def test_md_sync_check_overflow(c1):
    s = c1
    prm = params_of(s)
    x, v = dev(s.x), dev(s.v)
    f = torch.zeros_like(x)
    nl = api.NeighborList(s.n, 30, s.box, prm)
    with pytest.raises(L.LjmdError) as e:
        api.md_step(x, v, f, None, s.box, prm, nl, s.dt, 40, setup=True, sync_check=True)
    assert e.value.code == L.ENEIGH_OVERFLOW


# ---------------------------------------------------------------- adjoint


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("case", ["c1", "binary2k", "binary500"])
def test_backward_vs_oracle(oracle, case, fmt, c1, binary2k, binary500):
    s = {"c1": c1, "binary2k": binary2k, "binary500": binary500}[case]
    x = dev(s.x)
    prm = params_of(s)
    t = types_of(s)
    nl = api.build_list(x, t, s.box, prm, global_format=fmt == "global")
    g = np.random.default_rng(7).normal(size=(s.n, 3))
    gx, geps, gsig = api.lj_backward(x, t, s.box, prm, nl, dev(g))
    rx, re, rs = oracle.backward_brute(oracle.wrap(s.x, s.box), s.types, s.box, s.eps, s.sigma,
                                       s.rc, g)
    assert rel_err(gx.cpu().numpy(), rx) < 1e-11
    assert rel_err(geps.cpu().numpy(), re) < 1e-11
    assert rel_err(gsig.cpu().numpy(), rs) < 1e-11


@pytest.mark.parametrize("lanes", [0, 1, 2, 4, 8])
@pytest.mark.parametrize("case", ["binary2k", "large_cells"])
def test_backward_lanes_and_chunks(oracle, gather_lanes, case, lanes, binary2k):
    """The tiled adjoint with 1, 2, 4 or 8 lanes per atom, or chosen per tile
    (0), against the FP64 oracle.  large_cells (about 420 atoms per cell,
    single type, rc 7) has stencils many times larger than the adjoint's LDS
    stage, so every row is walked chunk by chunk with its per-lane cursor."""
    if case == "large_cells":
        x0, box = inputs.random_sites(27000, 1.0, seed=23)
        eps, sig, rc = inputs.single_type_tables(rc=7.0)
        prm = api.LJParams(eps=eps, sigma=sig, rc=rc, skin=0.3)
        types, t = None, None
    else:
        s = binary2k
        x0, box, prm, types, t = s.x, s.box, params_of(s), s.types, types_of(s)
        eps, sig, rc = s.eps, s.sigma, s.rc
    x = dev(x0)
    nl = api.build_list(x, t, box, prm)
    assert nl.format == "tiled"
    api.set_gather_lanes(lanes)
    g = np.random.default_rng(5).normal(size=(x0.shape[0], 3))
    gx, geps, gsig = api.lj_backward(x, t, box, prm, nl, dev(g))
    rx, re, rs = oracle.backward_cells(oracle.wrap(x0, box), types, box, eps, sig, rc, g)
    assert rel_err(gx.cpu().numpy(), rx) < 1e-11
    assert rel_err(geps.cpu().numpy(), re) < 1e-11
    assert rel_err(gsig.cpu().numpy(), rs) < 1e-11
    gx2, _, _ = api.lj_backward(x, t, box, prm, nl, dev(g))
    assert torch.equal(gx, gx2)


@pytest.mark.parametrize("fmt", ["tiled", "global"])
@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("case", ["c1", "binary2k"])
def test_fm_grad_equals_composed(oracle, case, mixed, fmt, c1, binary2k):
    """ljmd_fm_grad (forces, loss gradient written by the gather as each force
    completes, adjoint) against lj_forces, g = (F - F_t) * (2/n), lj_backward:
    bit for bit; the FP64 one also against the oracle's gradient of the mean
    squared force error, and an explicit weight against the default one."""
    s = {"c1": c1, "binary2k": binary2k}[case]
    x = dev(s.x)
    t = types_of(s)
    prm = params_of(s)
    nl = api.build_list(x, t, s.box, prm, global_format=fmt == "global")
    ft = dev(np.random.default_rng(41).normal(size=(s.n, 3)))
    f, _ = api.lj_forces(x, t, s.box, prm, nl, mixed=mixed)
    ref = api.lj_backward(x, t, s.box, prm, nl, (f - ft) * (2.0 / s.n))
    f2 = torch.full_like(f, float("nan"))
    got = api.fm_grad(x, t, s.box, prm, nl, ft, mixed=mixed, f=f2)
    assert torch.equal(f, f2)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    w = torch.tensor([2.0 / s.n], dtype=torch.float64, device=DEV)
    got_w = api.fm_grad(x, t, s.box, prm, nl, ft, weight=w, mixed=mixed)
    for a, b in zip(ref, got_w):
        assert torch.equal(a, b)
    if not mixed:
        xw = oracle.wrap(s.x, s.box)
        fr, _ = oracle.forces_brute(xw, s.types, s.box, s.eps, s.sigma, s.rc)
        rx, re, rs = oracle.backward_brute(xw, s.types, s.box, s.eps, s.sigma, s.rc,
                                           (fr - ft.cpu().numpy()) * (2.0 / s.n))
        assert rel_err(got[0].cpu().numpy(), rx) < 1e-11


def test_adjoint_graph_replay(binary2k):
    """Forward forces, loss gradient and adjoint captured in one HIP graph:
    every replay (with eager work and synchronizations in between) gives the
    eager gradients bit for bit."""
    s = binary2k
    prm = params_of(s)
    x, t = dev(s.x), types_of(s)
    nl = api.build_list(x, t, s.box, prm)
    ws = api.workspace(s.n, s.box, prm)
    e_t, s_t = inputs.perturbed_params(s.eps, s.sigma, seed=4)
    ft, _ = api.lj_forces(x, t, s.box, api.LJParams(e_t, s_t, s.rc, s.skin), nl)
    f, g = torch.empty_like(x), torch.empty_like(x)

    def grad():
        api.lj_forces(x, t, s.box, prm, nl, f=f, ws=ws)
        torch.sub(f, ft, out=g).mul_(2.0 / s.n)
        return api.lj_backward(x, t, s.box, prm, nl, g, ws=ws)

    ref = [r.clone() for r in grad()]
    graph = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(graph, stream=st):
            out = grad()
    torch.cuda.current_stream().wait_stream(st)
    for _ in range(4):
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(out, ref):
            assert torch.equal(a, b)
        eager = grad()
        torch.cuda.synchronize()
        for a, b in zip(eager, ref):
            assert torch.equal(a, b)


def test_autograd_force_matching(oracle, binary2k):
    """loss = (1/N) sum |F - F_t|^2 through LJForce; gradients equal the oracle's
    adjoint with g = 2 (F - F_t) / N."""
    from paper_2508_13523_amd.autograd import LJForce

    s = binary2k
    t = types_of(s)
    prm = params_of(s)
    x = dev(s.x)
    nl = api.build_list(x, t, s.box, prm)
    e_t, s_t = inputs.perturbed_params(s.eps, s.sigma, seed=4)
    xw = oracle.wrap(s.x, s.box)
    ft, _ = oracle.forces_brute(xw, s.types, s.box, e_t, s_t, s.rc)
    eps = torch.tensor(s.eps, requires_grad=True)
    sig = torch.tensor(s.sigma, requires_grad=True)
    xg = x.clone().requires_grad_(True)
    ws = api.workspace(s.n, s.box, prm)
    F = LJForce.apply(xg, eps, sig, (t, s.box, s.rc, s.skin, nl, ws))
    loss = ((F - dev(ft)) ** 2).sum() / s.n
    loss.backward()
    f_ref, _ = oracle.forces_brute(xw, s.types, s.box, s.eps, s.sigma, s.rc)
    g = 2.0 * (f_ref - ft) / s.n
    rx, re, rs = oracle.backward_brute(xw, s.types, s.box, s.eps, s.sigma, s.rc, g)
    assert rel_err(xg.grad.cpu().numpy(), rx) < 1e-10
    assert rel_err(eps.grad.numpy(), re) < 1e-10
    assert rel_err(sig.grad.numpy(), rs) < 1e-10
    # the same through the unique type-pair parameters (AA, AB, BB)
    from paper_2508_13523_amd.autograd import pair_table
    ue = torch.tensor([s.eps[0, 0], s.eps[0, 1], s.eps[1, 1]], requires_grad=True)
    us = torch.tensor([s.sigma[0, 0], s.sigma[0, 1], s.sigma[1, 1]], requires_grad=True)
    F = LJForce.apply(x.clone(), pair_table(ue, 2), pair_table(us, 2),
                      (t, s.box, s.rc, s.skin, nl, ws))
    (((F - dev(ft)) ** 2).sum() / s.n).backward()
    for got, tab in ((ue.grad.numpy(), re), (us.grad.numpy(), rs)):
        want = np.array([tab[0, 0], tab[0, 1] + tab[1, 0], tab[1, 1]])
        assert rel_err(got, want) < 1e-10


# ---------------------------------------------------------------- full sizes


@pytest.fixture(scope="module")
def c2():
    return inputs.fcc_liquid(40)  # 256,000 atoms


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("mode", ["full", "half"])
def test_c2_256k(oracle, c2, mode, fmt):
    s = c2
    x = dev(s.x)
    prm = params_of(s)
    nl = api.build_list(x, None, s.box, prm, mode=mode, global_format=fmt == "global")
    assert nl.format == fmt
    assert_list_equal(nl.to_csr(), oracle.nl_cells(s.x, None, s.box, s.rc, s.skin, mode == "half"),
                      mode == "half")
    f, ev = api.lj_forces(x, None, s.box, prm, nl, ev=True)
    f_ref, ev_ref = oracle.forces_cells(oracle.wrap(s.x, s.box), None, s.box, s.eps, s.sigma, s.rc)
    assert rel_err(f.cpu().numpy(), f_ref) < 1e-12
    check_ev(ev.cpu().numpy(), ev_ref)


@pytest.fixture(scope="module")
def c3():
    return inputs.fcc_liquid(80)  # 2,048,000 atoms


def sampled_parity(oracle, s, nrows, seed, sort):
    """Sampled parity at full size: the full-list build (tiled), the FP64 and
    mixed gathers, against brute-force oracle rows of `nrows` random atoms
    plus the first and last; with `sort` the atoms are first put into cell
    order by md_step (as the benchmark runs them) and the outputs are mapped
    back to the input order through the permuted ids."""
    x = dev(s.x)
    prm = params_of(s)
    xw = oracle.wrap(s.x, s.box)
    if sort:
        ids = torch.arange(s.n, dtype=torch.int32, device=DEV)
        nl = api.NeighborList(s.n, api.default_capacity(prm, s.box, s.n), s.box, prm)
        api.md_step(x, dev(s.v), torch.zeros_like(x), None, s.box, prm, nl, s.dt, 0,
                    setup=True, sort=True, ids=ids)
        assert api.get_status(nl)[L.ST_OVERFLOW] == 0
        perm = ids.cpu().numpy().astype(np.int64)  # position k holds input atom perm[k]
        assert np.array_equal(np.sort(perm), np.arange(s.n))
    else:
        nl = api.build_list(x, None, s.box, prm, mode="full")
        perm = np.arange(s.n)
    assert nl.format == "tiled"
    assert np.array_equal(x.cpu().numpy(), xw[perm])
    where = np.empty(s.n, dtype=np.int64)
    where[perm] = np.arange(s.n)  # input atom -> position
    rows = np.random.default_rng(seed).choice(s.n, nrows, replace=False)
    rows = np.concatenate([rows, [0, s.n - 1]])

    def user_rows(r_user):
        counts, off, idx, _ = nl.rows_csr(where[r_user])
        idx = perm[idx]
        out = np.concatenate([np.sort(idx[off[k]:off[k + 1]]) for k in range(len(r_user))]) \
            if len(idx) else idx
        return counts, off, out

    counts, off, idx = user_rows(rows)
    rc_, ro, ri = oracle.nl_rows(s.x, None, s.box, s.rc, s.skin, rows)
    assert np.array_equal(counts, rc_) and np.array_equal(idx, ri)
    # symmetry: every partner's row lists the sampled atom
    partners = np.unique(idx)
    pc, po, pi = user_rows(partners)
    at = {int(j): k for k, j in enumerate(partners)}
    for k, i in enumerate(rows):
        for j in idx[off[k]:off[k + 1]]:
            q = at[int(j)]
            assert i in pi[po[q]:po[q + 1]]
    fr = oracle.force_rows(xw, None, s.box, s.eps, s.sigma, s.rc, rows)
    out = {}
    for mixed in (False, True):
        f, _ = api.lj_forces(x, None, s.box, prm, nl, mixed=mixed)
        fh = f.cpu().numpy()
        got = fh[where[rows]]
        if mixed:
            out["mixed_worst"] = check_mixed(got, None, fr, None, xw, None, s.box, s.eps,
                                             s.sigma, s.rc, (rc_, ro, ri), rows=rows)
        else:
            assert np.abs(got - fr).max() / np.abs(fr).max() < 1e-12
        # Newton's third law over the whole system
        assert np.abs(fh.sum(axis=0)).max() < 1e-9 * np.abs(fh).max() * math.sqrt(s.n)
    return out


def test_c3_2M_sampled(oracle, c3):
    """At the benchmarked size (2,048,000 atoms, full list, gather): 192 sampled
    rows and forces against brute-force oracle rows, plus properties that hold
    at any size (sum of forces, list symmetry on the sampled rows); atoms in
    the input order (the cell-order lookup of the build and gather)."""
    sampled_parity(oracle, c3, 192, 11, sort=False)


def test_c3_2M_sampled_sorted(oracle, c3):
    """The same at 2,048,000 atoms with the atoms in cell order, as the
    benchmark's MD keeps them."""
    out = sampled_parity(oracle, c3, 96, 13, sort=True)
    print(f"2M sorted: mixed max |dF_i|/S_i = {out['mixed_worst']:.3e}")


def test_c3_16M_sampled(oracle):
    """16,384,000 atoms (160^3 FCC cells, the larger single-GPU size of the
    LJ comparison): 64 sampled rows plus the first and last, atoms in cell
    order as in the benchmark; lists bit-exact, FP64 forces within 1e-12,
    mixed forces within their rounding bound, Newton's third law overall."""
    s = inputs.fcc_liquid(160)
    assert s.n == 16_384_000
    out = sampled_parity(oracle, s, 64, 17, sort=True)
    print(f"16M sorted: mixed max |dF_i|/S_i = {out['mixed_worst']:.3e}")
