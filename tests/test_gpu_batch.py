"""GPU parity of the batch path (many independent systems per launch) against
the CPU oracle run on each system alone, for both batch list formats (tiled:
one workgroup per tile of every system; global: batch-wide atom indices).

Bars as for one system: lists bit-exact as sets per system, FP64 forces,
energies and virials within 1e-12, mixed precision within the rounding bound
of its FP32 pair terms (tests/mixed_bound.py) and 2e-6 normwise, adjoint
within 1e-11, trajectories within 1e-9.  Every force-kernel variant
the autotuner can pick gives the same forces within 1e-12, and a captured
HIP graph of the MD step reproduces the eager run bit for bit on every
replay.
"""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2508_13523_amd import _lib as L
from paper_2508_13523_amd import api, batch as B, inputs

from mixed_bound import check_mixed

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda"
# uneven sizes; 500 and 600 atoms give boxes with 2 cells per dimension
SIZES = [500, 1300, 600, 2500, 900, 3100, 700]
TUNINGS = [(l, b, p) for l in (0, 1, 2, 4) for b in (128, 256) for p in (0, 4, 8)]
FMTS = ["tiled", "global"]


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def rel_err(a, b):
    scale = np.abs(b).max()
    return np.abs(a - b).max() / (scale if scale > 0 else 1.0)


@pytest.fixture(scope="module")
def rb():
    return inputs.replica_batch(SIZES, seed_base=2000)


def setup_batch(rb):
    bt = B.Batch(rb["offsets"], rb["boxes"])
    prm = api.LJParams(rb["eps"], rb["sigma"], rb["rc"], rb["skin"], rb["mass"])
    return bt, prm, dev(rb["x"]), dev(rb["types"], torch.int32)


@pytest.mark.parametrize("fmt", FMTS)
def test_batch_lists_match_each_system(oracle, rb, fmt):
    bt, prm, x, t = setup_batch(rb)
    nl = B.build_list(x, t, bt, prm, global_format=fmt == "global")
    assert nl.format == fmt and nl.c().flags & L.NL_BATCH
    counts, offsets, idx, codes = nl.to_csr()
    xw = x.cpu().numpy()
    for r, s in enumerate(rb["systems"]):
        sl = bt.system(r)
        assert np.array_equal(xw[sl], oracle.wrap(s.x, s.box))
        rc_, ro, ri = oracle.nl_cells(s.x, s.types, s.box, s.rc, s.skin, False)
        c = counts[sl]
        assert np.array_equal(c, rc_), r
        got = idx[offsets[sl.start]:offsets[sl.stop]]
        assert np.array_equal(got - sl.start, ri), r


@pytest.mark.parametrize("fmt", FMTS)
def test_batch_forces_fp64_and_ev(oracle, rb, fmt):
    bt, prm, x, t = setup_batch(rb)
    nl = B.build_list(x, t, bt, prm, global_format=fmt == "global")
    f, ev = B.lj_forces(x, t, bt, prm, nl, ev=True)
    f, ev = f.cpu().numpy(), ev.cpu().numpy()
    for r, s in enumerate(rb["systems"]):
        fr, evr = oracle.forces_cells(oracle.wrap(s.x, s.box), s.types, s.box, s.eps, s.sigma,
                                      s.rc)
        assert rel_err(f[bt.system(r)], fr) < 1e-12, r
        assert np.abs(ev[r] - evr).max() <= 1e-12 * np.abs(evr).max(), r


def stretched_batch(specs):
    """Binary-liquid systems (n, seed, density, stretch along x), each box and
    its positions stretched along x after the start is drawn: dilute,
    elongated systems whose grid rows are long and whose cells hold few atoms."""
    systems = []
    for n, seed, rho, sx in specs:
        sy = inputs.binary_liquid(n, seed, rho=rho)
        k = np.array([sx, 1.0, 1.0])
        systems.append(dataclasses.replace(sy, x=sy.x * k, box=sy.box * k))
    off = np.zeros(len(systems) + 1, dtype=np.int64)
    np.cumsum([sy.n for sy in systems], out=off[1:])
    s0 = systems[0]
    return dict(x=np.concatenate([sy.x for sy in systems]),
                v=np.concatenate([sy.v for sy in systems]),
                types=np.concatenate([sy.types for sy in systems]), offsets=off,
                boxes=np.stack([sy.box for sy in systems]), eps=s0.eps, sigma=s0.sigma,
                rc=s0.rc, skin=s0.skin, mass=s0.mass, systems=systems)


def test_batch_tiles_at_table_limits(oracle):
    """Tiled batch lists whose tiles reach the tile tables' limits: grid rows
    of 21 and 26 cells (strips of the whole row; the staged-cell limit leaves
    2 and 1 rows along y: 276 and 252 of 288 staged cells), a dilute cube
    whose tiles are 7 x 7 cells (27 staged rows), and a dense system.  Lists
    bit-exact as sets, FP64 forces and energy/virial, and the adjoint,
    against the oracle system by system."""
    sb = stretched_batch([(2000, 41, 0.6, 4.0), (2000, 43, 0.3, 4.0), (1600, 47, 0.2, 1.0),
                          (900, 53, 1.2, 1.0)])
    bt, prm, x, t = setup_batch(sb)
    nl = B.build_list(x, t, bt, prm)
    assert nl.format == "tiled"
    counts, offsets, idx, _ = nl.to_csr()
    f, ev = B.lj_forces(x, t, bt, prm, nl, ev=True)
    f, ev = f.cpu().numpy(), ev.cpu().numpy()
    g = np.random.default_rng(29).normal(size=(bt.n, 3))
    gx, _, _ = B.lj_backward(x, t, bt, prm, nl, dev(g))
    gx = gx.cpu().numpy()
    for r, sy in enumerate(sb["systems"]):
        sl = bt.system(r)
        rc_, _, ri = oracle.nl_cells(sy.x, sy.types, sy.box, sy.rc, sy.skin, False)
        assert np.array_equal(counts[sl], rc_), r
        assert np.array_equal(idx[offsets[sl.start]:offsets[sl.stop]] - sl.start, ri), r
        xw = oracle.wrap(sy.x, sy.box)
        fr, evr = oracle.forces_cells(xw, sy.types, sy.box, sy.eps, sy.sigma, sy.rc)
        assert rel_err(f[sl], fr) < 1e-12, r
        assert np.abs(ev[r] - evr).max() <= 1e-12 * np.abs(evr).max(), r
        rx, _, _ = oracle.backward_cells(xw, sy.types, sy.box, sy.eps, sy.sigma, sy.rc, g[sl])
        assert rel_err(gx[sl], rx) < 1e-11, r


@pytest.mark.parametrize("fmt", FMTS)
def test_batch_forces_mixed(oracle, rb, fmt):
    bt, prm, x, t = setup_batch(rb)
    nl = B.build_list(x, t, bt, prm, global_format=fmt == "global")
    f, ev = B.lj_forces(x, t, bt, prm, nl, mixed=True, ev=True)
    f, ev = f.cpu().numpy(), ev.cpu().numpy()
    for r, s in enumerate(rb["systems"]):
        xw = oracle.wrap(s.x, s.box)
        fr, evr = oracle.forces_cells(xw, s.types, s.box, s.eps, s.sigma, s.rc)
        csr = oracle.nl_cells(s.x, s.types, s.box, s.rc, 0.0)
        check_mixed(f[bt.system(r)], ev[r], fr, evr, xw, s.types, s.box, s.eps, s.sigma, s.rc,
                    csr)


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("mixed", [False, True])
def test_batch_every_tuning_agrees(rb, mixed, fmt):
    bt, prm, x, t = setup_batch(rb)
    nl = B.build_list(x, t, bt, prm, global_format=fmt == "global")
    B.set_tuning(bt, prm, None, mixed)
    f0, _ = B.lj_forces(x, t, bt, prm, nl, mixed=mixed)
    f0 = f0.cpu().numpy()
    for tun in TUNINGS:
        B.set_tuning(bt, prm, tun, mixed)
        f, _ = B.lj_forces(x, t, bt, prm, nl, mixed=mixed)
        assert rel_err(f.cpu().numpy(), f0) < 1e-12, tun
    best = B.autotune(x, t, bt, prm, nl, mixed=mixed)
    assert best[:3] in TUNINGS and best[3] == 300
    if fmt == "tiled":  # variants by lane count and persistence
        assert best[1] == 256
    f, _ = B.lj_forces(x, t, bt, prm, nl, mixed=mixed)
    assert rel_err(f.cpu().numpy(), f0) < 1e-12
    B.set_tuning(bt, prm, None, mixed)
    with pytest.raises(L.LjmdError):
        B.set_tuning(bt, prm, (3, 256, 0), mixed)


TILE_TARGETS = [150, 200, 300, 450, 600]


def test_batch_tile_targets_match_oracle(oracle, rb):
    """Every tile target the autotuner searches: the tiled batch list built
    for it is bit-exact per system, FP64 forces, energies and virials within
    1e-12, the FP64 adjoint within 1e-11 of the oracle; a list is refused by
    a batch that names another target; the tile search picks one of them,
    leaves the list built for it and the forces unchanged."""
    _, prm, x0, t = setup_batch(rb)
    g = np.random.default_rng(11).normal(size=(x0.shape[0], 3))
    refs = []
    for r, s in enumerate(rb["systems"]):
        xw = oracle.wrap(s.x, s.box)
        fr, evr = oracle.forces_cells(xw, s.types, s.box, s.eps, s.sigma, s.rc)
        refs.append((fr, evr, oracle.nl_cells(s.x, s.types, s.box, s.rc, s.skin, False)))
    f_first = None
    for target in TILE_TARGETS:
        bt = B.Batch(rb["offsets"], rb["boxes"], tile_atoms=target)
        x = x0.clone()
        nl = B.build_list(x, t, bt, prm)
        assert nl.format == "tiled" and nl.tile[0] == target
        counts, offsets, idx, _ = nl.to_csr()
        f, ev = B.lj_forces(x, t, bt, prm, nl, ev=True)
        gx, _, _ = B.lj_backward(x, t, bt, prm, nl, dev(g))
        f, ev, gx = f.cpu().numpy(), ev.cpu().numpy(), gx.cpu().numpy()
        for r, s in enumerate(rb["systems"]):
            sl = bt.system(r)
            fr, evr, (rc_, ro, ri) = refs[r]
            assert np.array_equal(counts[sl], rc_), (target, r)
            base = sl.start
            for k in range(s.n):
                a = base + k
                row = np.sort(idx[offsets[a]:offsets[a + 1]] - base)
                assert np.array_equal(row, ri[ro[k]:ro[k + 1]]), (target, r, k)
            assert rel_err(f[sl], fr) < 1e-12, (target, r)
            assert np.abs(ev[r] - evr).max() <= 1e-12 * np.abs(evr).max(), (target, r)
            rx, _, _ = oracle.backward_cells(oracle.wrap(s.x, s.box), s.types, s.box, s.eps,
                                             s.sigma, s.rc, g[sl])
            assert rel_err(gx[sl], rx) < 1e-11, (target, r)
        if f_first is None:
            f_first = f
        # a batch naming another tile target refuses the list
        other = B.Batch(rb["offsets"], rb["boxes"], tile_atoms=target + 1)
        with pytest.raises(L.LjmdError):
            B.lj_forces(x, t, other, prm, nl)
    bt = B.Batch(rb["offsets"], rb["boxes"])
    x = x0.clone()
    nl = B.build_list(x, t, bt, prm)
    for for_md in (False, True):
        best = B.autotune(x, t, bt, prm, nl, mixed=False, tiles=True, for_md=for_md)
        assert best[3] in TILE_TARGETS and bt.tile_atoms == best[3] and nl.tile[0] == best[3]
        f, _ = B.lj_forces(x, t, bt, prm, nl)
        assert rel_err(f.cpu().numpy(), f_first) < 1e-12
        B.set_tuning(bt, prm, None, False)


def test_batch_tiled_persistent_walk_equals_one_workgroup_per_tile():
    """A tiled batch list with about 1,200 tiles, so that persistent grids of
    2 or 4 workgroups per compute unit (512 or 1,024 workgroups) walk
    several tiles each: forces and energy/virial bit for bit equal to one
    workgroup per tile, at every lane setting."""
    sizes = inputs.replica_sizes(60, lo=2000, hi=6000, seed=17)
    big = inputs.replica_batch(sizes, seed_base=3000)
    bt, prm, x, t = setup_batch(big)
    nl = B.build_list(x, t, bt, prm)
    assert nl.format == "tiled"
    for mixed in (False, True):
        for lanes in (0, 1, 2, 4):
            B.set_tuning(bt, prm, (lanes, 256, 0), mixed)
            f0, ev0 = B.lj_forces(x, t, bt, prm, nl, mixed=mixed, ev=True)
            for pers in (2, 4):
                B.set_tuning(bt, prm, (lanes, 256, pers), mixed)
                f, ev = B.lj_forces(x, t, bt, prm, nl, mixed=mixed, ev=True)
                assert torch.equal(f, f0) and torch.equal(ev, ev0), (mixed, lanes, pers)
        B.set_tuning(bt, prm, None, mixed)


@pytest.mark.parametrize("fmt", FMTS)
def test_batch_backward(oracle, rb, fmt):
    bt, prm, x, t = setup_batch(rb)
    nl = B.build_list(x, t, bt, prm, global_format=fmt == "global")
    g = np.random.default_rng(11).normal(size=(bt.n, 3))
    gx, geps, gsig = B.lj_backward(x, t, bt, prm, nl, dev(g))
    gx = gx.cpu().numpy()
    se = np.zeros((2, 2))
    ss = np.zeros((2, 2))
    for r, s in enumerate(rb["systems"]):
        sl = bt.system(r)
        rx, re, rs = oracle.backward_cells(oracle.wrap(s.x, s.box), s.types, s.box, s.eps,
                                           s.sigma, s.rc, g[sl])
        assert rel_err(gx[sl], rx) < 1e-11, r
        se += re
        ss += rs
    assert rel_err(geps.cpu().numpy(), se) < 1e-11
    assert rel_err(gsig.cpu().numpy(), ss) < 1e-11


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("weighted", [False, True])
def test_batch_fm_grad_equals_composed(oracle, rb, fmt, mixed, weighted):
    """The one-call force-matching gradient (the gather writes the loss
    gradient g = w_r (F - F_target) as each force completes) against the
    composed path (batch forces, g formed on the host side, batch adjoint):
    forces, gx, geps and gsig bit for bit; with the default weights
    w_r = 2 / N_r also against the oracle's FP64 gradient of each system's
    mean squared force error (FP64 forward)."""
    bt, prm, x, t = setup_batch(rb)
    nl = B.build_list(x, t, bt, prm, global_format=fmt == "global")
    ft = dev(np.random.default_rng(12).normal(size=(bt.n, 3)))
    sizes = np.diff(np.asarray(rb["offsets"]))
    wr = (np.random.default_rng(13).uniform(0.5, 2.0, bt.nrep) if weighted
          else 2.0 / sizes.astype(np.float64))
    f, _ = B.lj_forces(x, t, bt, prm, nl, mixed=mixed)
    scale = dev(np.repeat(wr, sizes)[:, None])
    ref = B.lj_backward(x, t, bt, prm, nl, (f - ft) * scale)
    f2 = torch.full_like(f, float("nan"))
    got = B.fm_grad(x, t, bt, prm, nl, ft, weight=dev(wr) if weighted else None, mixed=mixed,
                    f=f2)
    assert torch.equal(f, f2)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    gx_nof = B.fm_grad(x, t, bt, prm, nl, ft, weight=dev(wr) if weighted else None,
                       mixed=mixed)[0]
    assert torch.equal(gx_nof, got[0])  # forces not written: same gradient
    if not mixed and not weighted:
        gx = got[0].cpu().numpy()
        ftn = ft.cpu().numpy()
        for r, s in enumerate(rb["systems"]):
            sl = bt.system(r)
            xw = oracle.wrap(s.x, s.box)
            fr, _ = oracle.forces_cells(xw, s.types, s.box, s.eps, s.sigma, s.rc)
            rx, _, _ = oracle.backward_cells(xw, s.types, s.box, s.eps, s.sigma, s.rc,
                                             (fr - ftn[sl]) * (2.0 / s.n))
            assert rel_err(gx[sl], rx) < 1e-11, r


def test_batch_backward_many_tiles(oracle):
    """The batch adjoint on a tiled list of about 1,200 tiles (60 systems of
    2,000-6,000 atoms, tiles several cells deep in y): positions and
    parameter gradients against the FP64 oracle, system by system."""
    sizes = inputs.replica_sizes(60, lo=2000, hi=6000, seed=17)
    big = inputs.replica_batch(sizes, seed_base=3000)
    bt, prm, x, t = setup_batch(big)
    nl = B.build_list(x, t, bt, prm)
    assert nl.format == "tiled"
    g = np.random.default_rng(12).normal(size=(bt.n, 3))
    gx, geps, gsig = B.lj_backward(x, t, bt, prm, nl, dev(g))
    gx = gx.cpu().numpy()
    se = np.zeros((2, 2))
    ss = np.zeros((2, 2))
    for r, s in enumerate(big["systems"]):
        sl = bt.system(r)
        rx, re, rs = oracle.backward_cells(oracle.wrap(s.x, s.box), s.types, s.box, s.eps,
                                           s.sigma, s.rc, g[sl])
        assert rel_err(gx[sl], rx) < 1e-11, r
        se += re
        ss += rs
    assert rel_err(geps.cpu().numpy(), se) < 1e-11
    assert rel_err(gsig.cpu().numpy(), ss) < 1e-11
    gx2, _, _ = B.lj_backward(x, t, bt, prm, nl, dev(g))
    assert np.array_equal(gx, gx2.cpu().numpy())


@pytest.mark.parametrize("fmt", FMTS)
def test_batch_md_matches_each_system(oracle, rb, fmt):
    bt, prm, x, t = setup_batch(rb)
    v = dev(rb["v"])
    f = torch.zeros_like(x)
    nl = B.neighbor_list(bt, prm, 192, global_format=fmt == "global")
    th = B.md_step(x, v, f, t, bt, prm, nl, 0.005, 40, rebuild_every=20, thermo_every=20,
                   setup=True, sync_check=True)
    th = th.cpu().numpy()
    assert th.shape == (3, bt.nrep, 9)
    xg, vg = x.cpu().numpy(), v.cpu().numpy()
    for r, s in enumerate(rb["systems"]):
        sl = bt.system(r)
        xr, vr, fr, thr = oracle.md(s.x, s.v, s.types, s.box, s.eps, s.sigma, s.rc, s.mass,
                                    0.005, 40, rebuild_every=20, thermo_every=20, skin=s.skin)
        assert np.abs(xg[sl] - xr).max() < 1e-9, r
        assert np.abs(vg[sl] - vr).max() < 1e-8, r
        assert np.allclose(th[:, r, :], thr, rtol=1e-9, atol=1e-9 * np.abs(thr).max()), r
    st = B.get_status(nl)
    assert st[L.ST_OVERFLOW] == 0 and st[L.ST_NONFINITE] == 0


@pytest.mark.parametrize("fmt", FMTS)
def test_batch_md_sorted_is_a_permutation(oracle, rb, fmt):
    """With atom sorting, atoms stay inside their own system and the state is
    the unsorted run's, permuted by the ids."""
    bt, prm, x, t = setup_batch(rb)
    v = dev(rb["v"])
    f = torch.zeros_like(x)
    ids = torch.arange(bt.n, dtype=torch.int32, device=DEV)
    nl = B.neighbor_list(bt, prm, 192, global_format=fmt == "global")
    B.md_step(x, v, f, t, bt, prm, nl, 0.005, 30, rebuild_every=10, setup=True, sort=True,
              ids=ids, mixed=False)
    x2, v2 = dev(rb["x"]), dev(rb["v"])
    f2 = torch.zeros_like(x2)
    nl2 = B.neighbor_list(bt, prm, 192, global_format=fmt == "global")
    t2 = dev(rb["types"], torch.int32)
    B.md_step(x2, v2, f2, t2, bt, prm, nl2, 0.005, 30, rebuild_every=10, setup=True)
    idn = ids.cpu().numpy()
    for r in range(bt.nrep):
        sl = bt.system(r)
        assert np.array_equal(np.sort(idn[sl]), np.arange(sl.start, sl.stop))
    assert np.abs(x.cpu().numpy() - x2.cpu().numpy()[idn]).max() < 1e-9
    assert np.array_equal(t.cpu().numpy(), rb["types"][idn])


@pytest.mark.parametrize("fmt", FMTS)
def test_batch_md_flags_unsafe_rebuild(rb, fmt):
    """The displacement check of each rebuild (half the skin, 0.15, since the
    last build) over a batch, 40 steps of dt = 0.0005 with a rebuild every 20:
    the atoms of the fresh start move at most 0.085 between rebuilds (the
    oracle's run of the same systems), so nothing is flagged; giving one
    system a uniform drift of 40 sigma/tau
    (its internal motion unchanged) moves its atoms 0.4 between rebuilds, and
    the list is flagged."""
    for boost, expect in ((0.0, 0), (40.0, 1)):
        bt, prm, x, t = setup_batch(rb)
        v = dev(rb["v"])
        v[bt.system(3), 0] += boost
        f = torch.zeros_like(x)
        nl = B.neighbor_list(bt, prm, 192, global_format=fmt == "global")
        B.md_step(x, v, f, t, bt, prm, nl, 0.0005, 40, rebuild_every=20, setup=True)
        st = B.get_status(nl)
        assert st[2] == expect and st[0] == 0 and st[3] == 0


def seeded_batch():
    """Six binary systems on jittered grids, each its own orthorhombic box and
    density (0.6 to 1.2; 2 to 7 cells per axis), in one batch."""
    rng = np.random.default_rng(77)
    systems = [inputs.grid_system(rng.integers(7, 17, size=3), rho, 40 + r, binary=True,
                                  jitter_std=0.05)
               for r, rho in enumerate([0.6, 1.2, 0.8442, 1.1, 0.7, 1.0])]
    off = np.zeros(len(systems) + 1, dtype=np.int64)
    np.cumsum([s.n for s in systems], out=off[1:])
    s0 = systems[0]
    return dict(x=np.concatenate([s.x for s in systems]), v=np.concatenate([s.v for s in systems]),
                types=np.concatenate([s.types for s in systems]), offsets=off,
                boxes=np.stack([s.box for s in systems]), eps=s0.eps, sigma=s0.sigma, rc=s0.rc,
                skin=s0.skin, mass=s0.mass, systems=systems)


@pytest.mark.parametrize("fmt", FMTS)
def test_batch_seeded_orthorhombic_systems(oracle, fmt):
    """Systems of different density and box shape in one batch: each
    system's list bit-exact, FP64 forces, energy and virial within 1e-12, and
    40 MD steps (dt = 0.002, from the far-from-equilibrium grid starts)
    within 1e-9 of the oracle's run of that system alone."""
    sb = seeded_batch()
    bt, prm, x, t = setup_batch(sb)
    nl = B.build_list(x, t, bt, prm, global_format=fmt == "global")
    assert nl.format == fmt
    counts, offsets, idx, _ = nl.to_csr()
    f, ev = B.lj_forces(x, t, bt, prm, nl, ev=True)
    f, ev = f.cpu().numpy(), ev.cpu().numpy()
    for r, s in enumerate(sb["systems"]):
        sl = bt.system(r)
        rc_, ro, ri = oracle.nl_cells(s.x, s.types, s.box, s.rc, s.skin, False)
        assert np.array_equal(counts[sl], rc_), r
        assert np.array_equal(idx[offsets[sl.start]:offsets[sl.stop]] - sl.start, ri), r
        fr, evr = oracle.forces_cells(oracle.wrap(s.x, s.box), s.types, s.box, s.eps, s.sigma,
                                      s.rc)
        assert rel_err(f[sl], fr) < 1e-12, r
        assert np.abs(ev[r] - evr).max() <= 1e-12 * np.abs(evr).max(), r
    x, v = dev(sb["x"]), dev(sb["v"])
    fm = torch.zeros_like(x)
    nl = B.neighbor_list(bt, prm, 256, global_format=fmt == "global")
    B.md_step(x, v, fm, t, bt, prm, nl, 0.002, 40, rebuild_every=10, setup=True, sync_check=True)
    xg = x.cpu().numpy()
    for r, s in enumerate(sb["systems"]):
        xr, vr, fr, _ = oracle.md(s.x, s.v, s.types, s.box, s.eps, s.sigma, s.rc, s.mass, 0.002,
                                  40, rebuild_every=10, skin=s.skin)
        assert np.abs(xg[bt.system(r)] - xr).max() < 1e-9, r
    st = B.get_status(nl)
    assert st[L.ST_OVERFLOW] == 0 and st[L.ST_NONFINITE] == 0


@pytest.mark.parametrize("sort", [False, True])
def test_batch_md_fused_kick_equals_separate(rb, sort):
    """With a tiled batch list the gather's epilogue runs the velocity-Verlet
    updates with the same fmas as the separate kick kernels: positions,
    velocities, forces, ids and thermo rows are bit-identical over 45 steps
    (rebuilds, thermo steps, odd and even step counts, two calls)."""
    bt, prm, _, _ = setup_batch(rb)
    runs = []
    for separate in (False, True):
        x, v, t = dev(rb["x"]), dev(rb["v"]), dev(rb["types"], torch.int32)
        f = torch.zeros_like(x)
        ids = torch.arange(bt.n, dtype=torch.int32, device=DEV)
        nl = B.neighbor_list(bt, prm, 192)
        th1 = B.md_step(x, v, f, t, bt, prm, nl, 0.005, 25, rebuild_every=10, thermo_every=5,
                        setup=True, sort=sort, ids=ids, separate_kick=separate)
        assert nl.format == "tiled"
        th2 = B.md_step(x, v, f, t, bt, prm, nl, 0.005, 20, step0=25, rebuild_every=10,
                        thermo_every=5, sort=sort, ids=ids, separate_kick=separate)
        runs.append((x, v, f, ids, torch.cat([th1, th2]), B.get_status(nl)))
    (xa, va, fa, ia, tha, sta), (xb, vb, fb, ib, thb, stb) = runs
    assert torch.equal(xa, xb) and torch.equal(va, vb) and torch.equal(fa, fb)
    assert torch.equal(ia, ib) and torch.equal(tha, thb)
    assert np.array_equal(sta, stb)


def test_batch_md_split_calls_any_parity(rb):
    """Batch MD with thermo steps (which only kick, so the fused update's
    position buffers change at the other steps): calls of 24 and 21 steps
    (an odd and an even number of buffer changes) equal one call of 45 steps
    bit for bit, thermo rows included."""
    bt, prm, _, _ = setup_batch(rb)
    runs = []
    for parts in ((45,), (24, 21)):
        x, v, t = dev(rb["x"]), dev(rb["v"]), dev(rb["types"], torch.int32)
        f = torch.zeros_like(x)
        nl = B.neighbor_list(bt, prm, 192)
        rows, step0 = [], 0
        for k, n in enumerate(parts):
            rows.append(B.md_step(x, v, f, t, bt, prm, nl, 0.005, n, step0=step0,
                                  rebuild_every=10, thermo_every=5, setup=k == 0, sort=True))
            step0 += n
        assert nl.format == "tiled"
        runs.append((x, v, f, torch.cat(rows)))
    (xa, va, fa, tha), (xb, vb, fb, thb) = runs
    assert torch.equal(xa, xb) and torch.equal(va, vb) and torch.equal(fa, fb)
    assert torch.equal(tha, thb)


@pytest.mark.parametrize("fmt", FMTS)
def test_batch_md_graph_replays_equal_eager(rb, fmt):
    """A HIP graph captured around the batch MD step (with a rebuild inside)
    reproduces the eager run on every replay, with eager work and
    synchronizations between the replays."""
    bt, prm, x0, t = setup_batch(rb)
    v0 = dev(rb["v"])
    f0 = torch.zeros_like(x0)
    nl = B.neighbor_list(bt, prm, 192, global_format=fmt == "global")
    ws = B.workspace(bt, prm)
    B.md_step(x0, v0, f0, t, bt, prm, nl, 0.005, 5, rebuild_every=20, setup=True, ws=ws)
    state0 = [a.clone() for a in (x0, v0, f0, nl.neigh, nl.numneigh, nl.aux, nl.xref)]
    thermo = torch.zeros((2, bt.nrep, 9), dtype=torch.float64, device=DEV)

    def restore():
        for dst, src in zip((x0, v0, f0, nl.neigh, nl.numneigh, nl.aux, nl.xref), state0):
            dst.copy_(src)

    # eager reference: steps 6 .. 25 (a rebuild at step 20, thermo at 10, 20)
    restore()
    B.md_step(x0, v0, f0, t, bt, prm, nl, 0.005, 20, step0=5, rebuild_every=20,
              thermo_every=10, ws=ws, thermo=thermo)
    torch.cuda.synchronize()
    ref = [a.clone() for a in (x0, v0, f0, thermo)]

    restore()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            B.md_step(x0, v0, f0, t, bt, prm, nl, 0.005, 20, step0=5, rebuild_every=20,
                      thermo_every=10, ws=ws, thermo=thermo)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        restore()
        thermo.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for got, want in zip((x0, v0, f0, thermo), ref):
            assert torch.equal(got, want), rep
        # eager work between replays
        B.lj_forces(x0, t, bt, prm, nl, ws=ws)
        torch.cuda.synchronize()


def test_bench_replicas_spot_parity(oracle):
    """The benchmark's 512-replica batch (N_r uniform on [500, 8000], seed 6,
    system r from seed 1000 + r, 2.19M atoms) run as the benchmark runs it:
    atoms put into cell order by the batch md_step, tiled list, the autotuned
    mixed forward and the FP64 adjoint.  Four systems -- the largest (6 cells
    per dimension), the smallest (2 cells per dimension) and two drawn at
    random -- against the oracle, outputs mapped back to the input order
    through the permuted ids: lists bit-exact, FP64 forces, energy and virial
    within 1e-12, mixed forces within their rounding bound, adjoint within
    1e-11."""
    sizes = inputs.replica_sizes(512, seed=6)
    rb = inputs.replica_batch(sizes, seed_base=1000)
    bt, prm, x, t = setup_batch(rb)
    v = dev(rb["v"])
    ids = torch.arange(bt.n, dtype=torch.int32, device=DEV)
    nl = B.build_list(x, t, bt, prm)
    ws = B.workspace(bt, prm)
    B.md_step(x, v, torch.empty_like(x), t, bt, prm, nl, 0.005, 0, setup=True, mixed=True,
              sort=True, ids=ids, ws=ws)
    assert nl.format == "tiled" and B.get_status(nl)[L.ST_OVERFLOW] == 0
    B.autotune(x, t, bt, prm, nl, mixed=True, ws=ws)
    f64, ev64 = B.lj_forces(x, t, bt, prm, nl, ev=True, ws=ws)
    fmx, evmx = B.lj_forces(x, t, bt, prm, nl, mixed=True, ev=True, ws=ws)
    perm = ids.cpu().numpy().astype(np.int64)
    g_user = np.random.default_rng(31).normal(size=(bt.n, 3))
    gx, _, _ = B.lj_backward(x, t, bt, prm, nl, dev(g_user[perm]), ws=ws)
    counts, offsets, idx, _ = nl.to_csr()
    xs, f64, fmx, gx = (a.cpu().numpy() for a in (x, f64, fmx, gx))
    ev64, evmx = ev64.cpu().numpy(), evmx.cpu().numpy()
    pick = [int(np.argmax(sizes)), int(np.argmin(sizes))]
    pick += [int(r) for r in np.random.default_rng(37).choice(512, 2, replace=False)]
    for r in pick:
        s = rb["systems"][r]
        sl = bt.system(r)
        pr = perm[sl] - sl.start  # position sl.start + k holds input atom pr[k]
        assert np.array_equal(np.sort(pr), np.arange(s.n)), r
        xw = oracle.wrap(s.x, s.box)
        assert np.array_equal(xs[sl], xw[pr]), r
        # list rows in input order, partners as input indices
        rc_, ro, ri = oracle.nl_cells(s.x, s.types, s.box, s.rc, s.skin, False)
        got_c = np.empty(s.n, dtype=np.int64)
        got_c[pr] = counts[sl]
        assert np.array_equal(got_c, rc_), r
        for k in range(s.n):
            a = sl.start + k
            row = np.sort(perm[idx[offsets[a]:offsets[a + 1]]] - sl.start)
            u = pr[k]
            assert np.array_equal(row, ri[ro[u]:ro[u + 1]]), (r, u)
        fr, evr = oracle.forces_cells(xw, s.types, s.box, s.eps, s.sigma, s.rc)
        f_user = np.empty_like(fr)
        f_user[pr] = f64[sl]
        assert rel_err(f_user, fr) < 1e-12, r
        assert np.abs(ev64[r] - evr).max() <= 1e-12 * np.abs(evr).max(), r
        fm_user = np.empty_like(fr)
        fm_user[pr] = fmx[sl]
        check_mixed(fm_user, evmx[r], fr, evr, xw, s.types, s.box, s.eps, s.sigma, s.rc,
                    oracle.nl_cells(s.x, s.types, s.box, s.rc, 0.0))
        rx, _, _ = oracle.backward_cells(xw, s.types, s.box, s.eps, s.sigma, s.rc,
                                         g_user[sl])
        gx_user = np.empty_like(rx)
        gx_user[pr] = gx[sl]
        assert rel_err(gx_user, rx) < 1e-11, r
    B.set_tuning(bt, prm, None, True)
