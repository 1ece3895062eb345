"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these checks re-call the oracle's own formula to produce an expected
value: they use closed-form special values of the 12-6 potential, its
scaling law, lattice sums over the FCC lattice (shell counts from the
textbook table in tests/golden/fcc_shells.txt, cross-checked by enumeration),
brute force, conservation laws, finite differences and an independent ODE
solver.
"""
import math
import os

import numpy as np
import pytest

from paper_2508_13523_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
RMIN = 2.0 ** (1.0 / 6.0)


def two_atoms(r, box=20.0, direction=(1.0, 0.0, 0.0)):
    u = np.asarray(direction, dtype=np.float64)
    u = u / np.linalg.norm(u)
    c = np.array([box / 2, box / 2, box / 2])
    x = np.stack([c - 0.5 * r * u, c + 0.5 * r * u])
    return x, np.full(3, box)


# ---------------------------------------------------------------- pair law


@pytest.mark.parametrize("eps,sig", [(1.0, 1.0), (1.5, 0.8), (0.5, 0.88), (2.0, 1.3)])
def test_pair_special_values(oracle, eps, sig):
    """U(sigma) = 0; U(2^(1/6) sigma) = -eps with zero force; |F(sigma)| = 24 eps/sigma
    (Sec. 4, Eq. (1))."""
    E, S, R = [[eps]], [[sig]], [[2.5 * sig]]
    x, box = two_atoms(sig)
    f, ev = oracle.forces_brute(x, None, box, E, S, R)
    assert abs(ev[0]) < 1e-13 * eps
    assert abs(np.linalg.norm(f[0]) - 24.0 * eps / sig) < 1e-12 * 24 * eps / sig
    # repulsive at r = sigma: atom 0 sits at smaller x, pushed towards -x
    assert f[0, 0] < 0 and f[1, 0] > 0
    x, box = two_atoms(RMIN * sig)
    f, ev = oracle.forces_brute(x, None, box, E, S, R)
    assert abs(ev[0] + eps) < 1e-14 * eps * 10
    assert np.abs(f).max() < 1e-13 * eps / sig * 24


def test_pair_scaling_law(oracle):
    """Dimensional analysis: U_{eps,sig}(r) = eps U_{1,1}(r/sig) and
    F_{eps,sig}(r) = (eps/sig) F_{1,1}(r/sig), for any r below the cutoff."""
    for eps, sig in [(1.5, 0.8), (0.5, 0.88), (3.0, 1.7)]:
        for s in [0.93, 1.0, 1.1, 1.4, 1.9, 2.3]:
            x1, b1 = two_atoms(s, box=30.0)
            f1, e1 = oracle.forces_brute(x1, None, b1, [[1.0]], [[1.0]], [[2.5]])
            x2, b2 = two_atoms(s * sig, box=30.0 * sig)
            f2, e2 = oracle.forces_brute(x2, None, b2, [[eps]], [[sig]], [[2.5 * sig]])
            # tolerance relative to the size of the two terms of the 12-6 law
            mag = 4.0 * eps * (s ** -12 + s ** -6)
            assert abs(e2[0] - eps * e1[0]) <= 1e-13 * mag
            # positions carry rounding of the box-centred placement (~1e-15 r), which
            # the steep force amplifies; scale by the size of the two force terms
            fmag = 24.0 * eps * (2 * s ** -13 + s ** -7) / sig
            assert np.allclose(f2, eps / sig * f1, rtol=0, atol=1e-13 * fmag)


def test_force_is_minus_energy_gradient_along_r(oracle):
    """U(r1) - U(r2) = integral_{r1}^{r2} |F|(r) dr (force/energy consistency),
    integrated with scipy's adaptive quadrature."""
    from scipy.integrate import quad

    def fr(r):
        x, box = two_atoms(r, box=30.0)
        f, _ = oracle.forces_brute(x, None, box, [[1.0]], [[1.0]], [[2.5]])
        return -f[0, 0]  # radial component on atom 1 = F . r_hat

    def u(r):
        x, box = two_atoms(r, box=30.0)
        return oracle.forces_brute(x, None, box, [[1.0]], [[1.0]], [[2.5]])[1][0]

    for r1, r2 in [(0.95, 1.3), (1.05, 2.0), (1.5, 2.45)]:
        integral, err = quad(fr, r1, r2, epsabs=1e-13, epsrel=1e-13)
        assert abs((u(r1) - u(r2)) - integral) < 1e-10


def test_cutoff_is_strict_and_unshifted(oracle):
    """Eq. (1) sums r < r_c only and has no energy shift: at r = r_c exactly the
    pair is absent, just inside it contributes U(r_c) = -0.0163..."""
    box = np.full(3, 20.0)
    x = np.array([[1.0, 5.0, 5.0], [3.5, 5.0, 5.0]])  # d = -2.5 exactly, rsq = 6.25
    f, ev = oracle.forces_brute(x, None, box, [[1.0]], [[1.0]], [[2.5]])
    assert ev[0] == 0.0 and np.all(f == 0.0)
    x[1, 0] = 3.5 - 1e-9
    f, ev = oracle.forces_brute(x, None, box, [[1.0]], [[1.0]], [[2.5]])
    u_rc = 4.0 * (2.5 ** -12 - 2.5 ** -6)
    assert abs(ev[0] - u_rc) < 1e-9 and ev[0] < 0
    x[1, 0] = 3.5 + 1e-9
    f, ev = oracle.forces_brute(x, None, box, [[1.0]], [[1.0]], [[2.5]])
    assert ev[0] == 0.0


def test_type_pair_indexing(oracle):
    """A pair of unlike types uses the [a][b] entry, in either order; like pairs use
    the diagonal.  Checked through U(sig_ab) = 0 and U(2^(1/6) sig_ab) = -eps_ab."""
    eps, sig, rc = inputs.binary_tables()
    for ta, tb, e, s in [(0, 1, 1.5, 0.8), (1, 0, 1.5, 0.8), (1, 1, 0.5, 0.88), (0, 0, 1.0, 1.0)]:
        t = np.array([ta, tb], dtype=np.int32)
        x, box = two_atoms(RMIN * s)
        f, ev = oracle.forces_brute(x, t, box, eps, sig, rc)
        assert abs(ev[0] + e) < 1e-13
        x, box = two_atoms(s)
        f, ev = oracle.forces_brute(x, t, box, eps, sig, rc)
        assert abs(ev[0]) < 1e-12
        assert abs(np.linalg.norm(f[0]) - 24 * e / s) < 1e-11


def test_minimum_image_across_boundary(oracle):
    """Two atoms 0.2 apart through the periodic boundary interact as a pair at 0.2,
    not at L - 0.2, in every dimension."""
    for dim in range(3):
        box = np.array([9.0, 10.0, 11.0])
        x = np.full((2, 3), 4.0)
        x[0, dim] = 0.1 + 1.0
        x[1, dim] = box[dim] - 0.1 - 0.0
        # separation through the boundary: 1.1 + 0.1 = 1.2
        f, ev = oracle.forces_brute(x, None, box, [[1.0]], [[1.0]], [[2.5]])
        xr, br = two_atoms(1.2)
        f2, ev2 = oracle.forces_brute(xr, None, br, [[1.0]], [[1.0]], [[2.5]])
        assert abs(ev[0] - ev2[0]) < 1e-13
        # atom 0 (near 0) is pushed/pulled along +dim in the same way atom 1 of the
        # reference pair is (its partner sits at its -dim side through the boundary)
        assert abs(f[0, dim] - f2[1, 0]) < 1e-12


# ---------------------------------------------------------------- lattice


def fcc_shells_golden():
    rows = []
    with open(os.path.join(HERE, "golden", "fcc_shells.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                m, c = line.split()
                rows.append((int(m), int(c)))
    return rows


def test_fcc_shell_table_matches_enumeration():
    """The golden shell counts agree with a direct enumeration of FCC lattice points."""
    counts = {}
    rng = range(-4, 5)
    for i in rng:
        for j in rng:
            for k in rng:
                for b in [(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]:
                    p = (2 * i + b[0], 2 * j + b[1], 2 * k + b[2])  # units of a/2
                    m2 = p[0] ** 2 + p[1] ** 2 + p[2] ** 2
                    if m2 == 0 or m2 % 2:
                        continue
                    counts[m2 // 2] = counts.get(m2 // 2, 0) + 1
    for m, c in fcc_shells_golden():
        assert counts.get(m, 0) == c


def lattice_sums(rho, rc, rnb):
    """E/N, (1/N) tr W and neighbor counts of a perfect FCC crystal, by shell sums."""
    a = (4.0 / rho) ** (1.0 / 3.0)
    e = w = 0.0
    n_rc = n_nb = 0
    for m, c in fcc_shells_golden():
        r = a * math.sqrt(m / 2.0)
        assert r > rnb or m < 12  # the table reaches beyond every cutoff used
        if r < rnb:
            n_nb += c
        if r < rc:
            n_rc += c
            e += 0.5 * c * 4.0 * (r ** -12 - r ** -6)
            # r . f(r) with f = -dU/dr:  r * 24 (2 r^-13 - r^-7)
            w += 0.5 * c * 24.0 * (2 * r ** -12 - r ** -6)
    return e, w, n_rc, n_nb


def test_perfect_fcc(oracle):
    """Perfect FCC at rho = 0.8442: 78 neighbors within 2.8, 54 within 2.5, zero
    force on every atom, and E/N, tr(W)/N equal to the shell sums."""
    x, box = inputs.fcc_lattice(5, inputs.RHO_FCC)
    n = x.shape[0]
    e_ref, w_ref, n_rc, n_nb = lattice_sums(inputs.RHO_FCC, 2.5, 2.8)
    assert (n_rc, n_nb) == (54, 78)
    assert abs(e_ref - (-6.7733680)) < 1e-6  # value quoted to 8 digits
    counts, _, _ = oracle.nl_brute(x, None, box, [[2.5]], 0.3)
    assert np.all(counts == 78)
    counts, _, _ = oracle.nl_brute(x, None, box, [[2.5]], 0.0)
    assert np.all(counts == 54)
    f, ev = oracle.forces_brute(x, None, box, [[1.0]], [[1.0]], [[2.5]])
    assert np.abs(f).max() < 1e-11
    assert abs(ev[0] / n - e_ref) < 1e-12 * abs(e_ref)
    assert abs((ev[1] + ev[2] + ev[3]) / n - w_ref) < 1e-12 * abs(w_ref)
    # cubic symmetry: diagonal virial components equal, off-diagonal vanish
    assert abs(ev[1] - ev[2]) < 1e-9 and abs(ev[1] - ev[3]) < 1e-9
    assert np.abs(ev[4:]).max() < 1e-9


# ---------------------------------------------------------------- systems


@pytest.fixture(scope="module")
def liquid():
    s = inputs.fcc_liquid(4)  # 256 atoms, L = 6.72
    return s


@pytest.fixture(scope="module")
def binary():
    return inputs.binary_liquid(600, seed=11)


def test_newton_third_law_and_invariances(oracle, liquid, binary):
    for s in (liquid, binary):
        f, ev = oracle.forces_brute(s.x, s.types, s.box, s.eps, s.sigma, s.rc)
        scale = np.abs(f).max()
        assert np.abs(f.sum(axis=0)).max() < 1e-12 * scale * math.sqrt(s.n)
        # translation invariance
        shift = np.array([0.37, -1.21, 2.05])
        f2, ev2 = oracle.forces_brute(inputs.into_box(s.x + shift, s.box), s.types, s.box,
                                      s.eps, s.sigma, s.rc)
        assert np.abs(f2 - f).max() < 1e-10 * scale
        assert abs(ev2[0] - ev[0]) < 1e-10 * abs(ev[0])
        # permutation equivariance
        p = np.random.default_rng(3).permutation(s.n)
        f3, ev3 = oracle.forces_brute(s.x[p], s.types[p], s.box, s.eps, s.sigma, s.rc)
        assert np.abs(f3 - f[p]).max() < 1e-11 * scale


def _near_cutoff(oracle, s, i, tol=1e-4):
    """True if atom i has a partner within tol of its pair cutoff."""
    counts, off, idx = oracle.nl_rows(s.x, s.types, s.box, s.rc, tol, [i])
    counts2, off2, idx2 = oracle.nl_rows(s.x, s.types, s.box, s.rc - tol, tol, [i])
    return counts[0] != counts2[0]


def test_force_is_minus_gradient_fd(oracle, liquid, binary):
    """F = -dE/dx by central differences, h = 1e-6, away from cutoff crossings."""
    rng = np.random.default_rng(5)
    h = 1e-6
    for s in (liquid, binary):
        f, _ = oracle.forces_brute(s.x, s.types, s.box, s.eps, s.sigma, s.rc)
        checked = 0
        for i in rng.choice(s.n, 24, replace=False):
            if _near_cutoff(oracle, s, i):
                continue
            for a in range(3):
                xp, xm = s.x.copy(), s.x.copy()
                xp[i, a] += h
                xm[i, a] -= h
                ep = oracle.forces_brute(xp, s.types, s.box, s.eps, s.sigma, s.rc)[1][0]
                em = oracle.forces_brute(xm, s.types, s.box, s.eps, s.sigma, s.rc)[1][0]
                fd = -(ep - em) / (2 * h)
                assert abs(fd - f[i, a]) < 1e-6 * max(1.0, abs(f[i, a])) + 2e-7 * abs(ep) / h * 1e-9
                checked += 1
        assert checked > 30


def test_virial_equals_cluster_moment(oracle):
    """For a cluster far from the periodic boundaries,
    W_ab = sum_{i<j} d_a (f_ij)_b = sum_i x_{i,a} F_{i,b}."""
    rng = np.random.default_rng(9)
    x, _ = inputs.random_sites(60, 1.0, seed=9, std=0.05)
    x = x + 20.0
    box = np.full(3, 60.0)
    eps, sig, rc = inputs.binary_tables()
    t = inputs.binary_types(60, 0.8, 4)
    f, ev = oracle.forces_brute(x, t, box, eps, sig, rc)
    m = x.T @ f  # m[a, b] = sum_i x_ia F_ib
    w = ev[1:]
    expect = [m[0, 0], m[1, 1], m[2, 2], m[0, 1], m[0, 2], m[1, 2]]
    scale = np.abs(m).max()
    assert np.allclose(w, expect, rtol=0, atol=1e-11 * scale)
    # the moment matrix is symmetric for central forces
    assert abs(m[0, 1] - m[1, 0]) < 1e-11 * scale
    del rng


# ---------------------------------------------------------------- neighbor lists


def _rows(counts, off, idx):
    return [tuple(idx[off[i]:off[i + 1]]) for i in range(len(counts))]


@pytest.mark.parametrize("case", ["fcc4", "binary600", "tiny2cell", "binary500"])
def test_neighbor_cells_equal_brute(oracle, case):
    """The cell-grid list equals the O(n^2) list, full and half, including boxes with
    2 cells per dimension (de-duplicated stencil)."""
    if case == "fcc4":
        s = inputs.fcc_liquid(4)
    elif case == "binary600":
        s = inputs.binary_liquid(600, seed=12)
    elif case == "binary500":
        s = inputs.binary_liquid(500, seed=13)  # L = 7.47: 2 cells per dim
    else:
        s = inputs.fcc_liquid(4, rho=1.1)  # L = 6.15: 2 cells per dim
    for half in (False, True):
        a = oracle.nl_brute(s.x, s.types, s.box, s.rc, s.skin, half)
        b = oracle.nl_cells(s.x, s.types, s.box, s.rc, s.skin, half)
        assert np.array_equal(a[0], b[0])
        assert np.array_equal(a[2], b[2])


def test_neighbor_list_symmetry_and_half(oracle, binary):
    s = binary
    counts, off, idx = oracle.nl_brute(s.x, s.types, s.box, s.rc, s.skin, False)
    full = _rows(counts, off, idx)
    pairs = {(i, j) for i, r in enumerate(full) for j in r}
    assert all((j, i) in pairs for (i, j) in pairs)
    assert all(i != j for (i, j) in pairs)
    hc, ho, hi = oracle.nl_brute(s.x, s.types, s.box, s.rc, s.skin, True)
    half = {(i, j) for i, r in enumerate(_rows(hc, ho, hi)) for j in r}
    assert half == {(i, j) for (i, j) in pairs if i < j}
    # rows of selected atoms equal the full rows
    rows = [0, 5, 77, s.n - 1]
    rc_, ro, ri = oracle.nl_rows(s.x, s.types, s.box, s.rc, s.skin, rows)
    for k, i in enumerate(rows):
        assert tuple(ri[ro[k]:ro[k + 1]]) == full[i]


def test_neighbor_hand_case(oracle):
    """Atoms 0 and 1 are 0.2 apart through the x boundary; atom 2 is 2.79 from
    atom 0 and sqrt(0.2^2 + 2.79^2) = 2.797 from atom 1 (both inside the 2.8
    neighbor cutoff); atom 3 is 2.81 from atom 1 and 2.817 from atom 0 (outside)."""
    box = np.array([10.0, 10.0, 10.0])
    x = np.array([[0.1, 5.0, 5.0], [9.9, 5.0, 5.0], [0.1, 7.79, 5.0], [9.9, 5.0, 7.81]])
    counts, off, idx = oracle.nl_brute(x, None, box, [[2.5]], 0.3)
    rows = _rows(counts, off, idx)
    assert rows[0] == (1, 2)
    assert rows[1] == (0, 2)
    assert rows[2] == (0, 1)
    assert rows[3] == ()


def test_wrap(oracle):
    box = np.array([5.0, 6.0, 7.0])
    x = np.array([[-1e-17, 6.0, 3.5], [5.0 - 1e-16, -0.25, 7.25]])
    w = oracle.wrap(x, box)
    assert np.all(w >= 0) and np.all(w < box)
    assert w[0, 0] == 0.0  # -1e-17 + 5 rounds to 5 -> mapped to 0
    assert w[0, 1] == 0.0 and w[1, 1] == 5.75 and w[1, 2] == 0.25


# ---------------------------------------------------------------- forces at scale


def test_forces_cells_equal_brute(oracle, liquid, binary):
    for s in (liquid, binary, inputs.binary_liquid(500, seed=2)):
        fa, ea = oracle.forces_brute(s.x, s.types, s.box, s.eps, s.sigma, s.rc)
        fb, eb = oracle.forces_cells(s.x, s.types, s.box, s.eps, s.sigma, s.rc)
        scale = np.abs(fa).max()
        assert np.abs(fa - fb).max() < 1e-12 * scale
        assert np.allclose(ea, eb, rtol=1e-12, atol=1e-12 * np.abs(ea).max())
        rows = np.array([0, 3, s.n // 2, s.n - 1])
        fr = oracle.force_rows(s.x, s.types, s.box, s.eps, s.sigma, s.rc, rows)
        assert np.abs(fr - fa[rows]).max() < 1e-12 * scale


# ---------------------------------------------------------------- integrator


def test_integrator_second_order_vs_ode_solver(oracle):
    """Two atoms released from rest at r0: velocity Verlet converges to the scipy
    DOP853 solution of the same Newton equations with error O(dt^2)."""
    from scipy.integrate import solve_ivp

    r0, tend = 1.6, 1.0

    def rhs(t, y):
        r = y[0]
        fmag = 24.0 * (2 * r ** -13 - r ** -7)  # -dU/dr of the unit pair
        return [y[1], 2.0 * fmag]  # reduced mass 1/2

    sol = solve_ivp(rhs, (0, tend), [r0, 0.0], method="DOP853", rtol=1e-13, atol=1e-13)
    r_exact = sol.y[0, -1]
    errs = []
    for dt in (0.01, 0.005, 0.0025):
        x, box = two_atoms(r0, box=30.0)
        v = np.zeros_like(x)
        steps = int(round(tend / dt))
        xf, vf, ff, _ = oracle.md(x, v, None, box, [[1.0]], [[1.0]], [[2.5]], [1.0], dt, steps,
                                  rebuild_every=10 ** 6)
        errs.append(abs(np.linalg.norm(xf[1] - xf[0]) - r_exact))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_integrator_time_reversible(oracle, liquid):
    s = liquid
    x1, v1, f1, th = oracle.md(s.x, s.v, s.types, s.box, s.eps, s.sigma, s.rc, s.mass, 0.005, 15,
                               rebuild_every=10 ** 6, thermo_every=5)
    x2, v2, f2, _ = oracle.md(x1, -v1, s.types, s.box, s.eps, s.sigma, s.rc, s.mass, 0.005, 15,
                              rebuild_every=10 ** 6, step0=15)
    d = x2 - s.x
    d -= s.box * np.round(d / s.box)  # the second run's set-up wraps into the box
    assert np.abs(d).max() < 1e-10
    assert np.abs(-v2 - s.v).max() < 1e-9
    # thermo rows: steps 0, 5, 10, 15; row values equal direct evaluation at the end
    assert list(th[:, 0]) == [0, 5, 10, 15]
    f, ev = oracle.forces_cells(x1, s.types, s.box, s.eps, s.sigma, s.rc)
    assert abs(th[-1, 1] - ev[0]) < 1e-12 * abs(ev[0])
    assert abs(th[-1, 2] - oracle.kinetic(v1, s.types, s.mass)) < 1e-12 * th[-1, 2]
    assert np.array_equal(th[-1, 3:], ev[1:])


def test_energy_conservation_is_second_order(oracle):
    """A cold FCC crystal (T = 0.02) never moves a pair across r_c (shells at 2.375 and
    2.656 straddle 2.5), so the total energy is smooth: its excursion stays small and
    shrinks about 4x when dt halves."""
    x, box = inputs.fcc_lattice(4)
    n = x.shape[0]
    v = inputs.maxwell(n, 0.02, np.ones(n), seed=3)
    dev = []
    for dt in (0.01, 0.005):
        steps = int(round(1.0 / dt))
        _, _, _, th = oracle.md(x, v, None, box, [[1.0]], [[1.0]], [[2.5]], [1.0], dt, steps,
                                rebuild_every=20, thermo_every=1)
        etot = (th[:, 1] + th[:, 2]) / n
        dev.append(np.abs(etot - etot[0]).max())
    assert dev[0] < 1e-4
    assert 3.0 < dev[0] / dev[1] < 5.0


def test_nve_liquid_energy_tracks_cutoff_crossings(oracle):
    """With the truncated, unshifted potential of Eq. (1) the total energy of a liquid
    changes only when pairs cross r_c, by U(r_c) each: over 200 steps from the jittered
    crystal, E_tot(t) - E_tot(0) equals U(r_c) times the change in the number of pairs
    inside r_c, up to the integrator's small error."""
    s = inputs.fcc_liquid(4)
    u_rc = 4.0 * (2.5 ** -12 - 2.5 ** -6)
    n0 = oracle.nl_brute(s.x, None, s.box, [[2.5]], 0.0, True)[0].sum()
    x, v, f, th = oracle.md(s.x, s.v, s.types, s.box, s.eps, s.sigma, s.rc, s.mass, 0.005, 200,
                            rebuild_every=20, thermo_every=20)
    n1 = oracle.nl_brute(x, None, s.box, [[2.5]], 0.0, True)[0].sum()
    etot = th[:, 1] + th[:, 2]
    assert n1 != n0
    assert abs((etot[-1] - etot[0]) - u_rc * (n1 - n0)) / s.n < 5e-4


def test_verlet_list_md_equals_exact_when_rebuilt_every_step(oracle, liquid):
    """The Verlet-list integrator (forces summed over a list of cutoff rc + skin,
    rebuilt every rebuild_every steps) is the exact pair sum when the list is
    rebuilt every step, and stays equal to it when the skin covers every
    approach between rebuilds."""
    s = liquid
    common = (s.types, s.box, s.eps, s.sigma, s.rc, s.mass, 0.005, 60)
    xe, ve, fe, te = oracle.md(s.x, s.v, *common, rebuild_every=1, thermo_every=10)
    xl, vl, fl, tl = oracle.md(s.x, s.v, *common, rebuild_every=1, thermo_every=10, skin=0.3)
    assert np.abs(xe - xl).max() < 1e-12 and np.abs(fe - fl).max() < 1e-10
    assert np.allclose(te, tl, rtol=1e-12, atol=1e-10)
    xe, ve, fe, te = oracle.md(s.x, s.v, *common, rebuild_every=20, thermo_every=10)
    xl, vl, fl, tl = oracle.md(s.x, s.v, *common, rebuild_every=20, thermo_every=10, skin=1.2)
    assert np.abs(xe - xl).max() < 1e-10


def test_verlet_list_md_misses_pairs_with_thin_skin(oracle):
    """With skin 0.3 and a rebuild every 20 steps at T = 1.44, some pairs close in
    from beyond rc + skin between rebuilds; the list-based run then departs
    from the exact pair sum (the method's truncation, not a rounding effect)."""
    s = inputs.fcc_liquid(5)
    common = (s.types, s.box, s.eps, s.sigma, s.rc, s.mass, 0.005, 100)
    xe, _, _, _ = oracle.md(s.x, s.v, *common, rebuild_every=20)
    xl, _, _, _ = oracle.md(s.x, s.v, *common, rebuild_every=20, skin=0.3)
    assert np.abs(xe - xl).max() > 1e-8


def test_maxwell_temperature(oracle):
    s = inputs.fcc_liquid(5)
    ke = oracle.kinetic(s.v, s.types, s.mass)
    assert abs(2 * ke / (3 * s.n - 3) - 1.44) < 1e-12
    assert np.abs(s.v.sum(axis=0)).max() < 1e-10


# ---------------------------------------------------------------- adjoint


def _loss(oracle, s, x, eps, sig, ft):
    f, _ = oracle.forces_brute(x, s.types, s.box, eps, sig, s.rc)
    return float(((f - ft) ** 2).sum() / s.n)


def test_adjoint_matches_finite_differences(oracle):
    """d/d(x, eps, sigma) of L = (1/N) sum |F - F_t|^2 from the oracle adjoint with
    g = 2 (F - F_t)/N, against central differences (h = 1e-6, cutoffs fixed)."""
    s = inputs.binary_liquid(300, seed=21)
    e_t, s_t = inputs.perturbed_params(s.eps, s.sigma, seed=4)
    ft, _ = oracle.forces_brute(s.x, s.types, s.box, e_t, s_t, s.rc)
    f, _ = oracle.forces_brute(s.x, s.types, s.box, s.eps, s.sigma, s.rc)
    g = 2.0 * (f - ft) / s.n
    gx, geps, gsig = oracle.backward_brute(s.x, s.types, s.box, s.eps, s.sigma, s.rc, g)
    assert np.allclose(geps, geps.T) and np.allclose(gsig, gsig.T)
    h = 1e-6
    L0 = _loss(oracle, s, s.x, s.eps, s.sigma, ft)
    rng = np.random.default_rng(5)
    checked = 0
    for i in rng.choice(s.n, 16, replace=False):
        if _near_cutoff(oracle, s, i):
            continue
        for a in range(3):
            xp, xm = s.x.copy(), s.x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = (_loss(oracle, s, xp, s.eps, s.sigma, ft) - _loss(oracle, s, xm, s.eps, s.sigma, ft)) / (2 * h)
            assert abs(fd - gx[i, a]) < 1e-6 * max(1.0, abs(gx[i, a])) + 1e-9 * abs(L0) / h
            checked += 1
    assert checked >= 30
    for a in range(2):
        for b in range(a, 2):
            for which in ("eps", "sig"):
                tp = (s.eps if which == "eps" else s.sigma).copy()
                tm = tp.copy()
                tp[a, b] += h
                tm[a, b] -= h
                if a != b:
                    tp[b, a] += h
                    tm[b, a] -= h
                args_p = (tp, s.sigma) if which == "eps" else (s.eps, tp)
                args_m = (tm, s.sigma) if which == "eps" else (s.eps, tm)
                fd = (_loss(oracle, s, s.x, *args_p, ft) - _loss(oracle, s, s.x, *args_m, ft)) / (2 * h)
                gt = geps if which == "eps" else gsig
                an = gt[a, b] + (gt[b, a] if a != b else 0.0)
                assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (which, a, b, fd, an)


def test_adjoint_is_symmetric_hessian_product(oracle):
    """backward(g = w) = -H w with H the (symmetric) Hessian of E:
    u . backward(w) = w . backward(u), and (F(x + h w) - F(x - h w)) / 2h = backward(w)."""
    s = inputs.binary_liquid(250, seed=31)
    rng = np.random.default_rng(8)
    u = rng.normal(size=(s.n, 3))
    w = rng.normal(size=(s.n, 3))
    bu = oracle.backward_brute(s.x, s.types, s.box, s.eps, s.sigma, s.rc, u)[0]
    bw = oracle.backward_brute(s.x, s.types, s.box, s.eps, s.sigma, s.rc, w)[0]
    lhs, rhs = float((u * bw).sum()), float((w * bu).sum())
    assert abs(lhs - rhs) < 1e-10 * max(abs(lhs), 1.0)
    h = 1e-6
    fp = oracle.forces_brute(s.x + h * w, s.types, s.box, s.eps, s.sigma, s.rc)[0]
    fm = oracle.forces_brute(s.x - h * w, s.types, s.box, s.eps, s.sigma, s.rc)[0]
    fd = (fp - fm) / (2 * h)
    assert np.abs(fd - bw).max() < 1e-5 * np.abs(bw).max()


def test_backward_cells_equal_brute(oracle):
    s = inputs.binary_liquid(500, seed=41)
    g = np.random.default_rng(1).normal(size=(s.n, 3))
    a = oracle.backward_brute(s.x, s.types, s.box, s.eps, s.sigma, s.rc, g)
    b = oracle.backward_cells(s.x, s.types, s.box, s.eps, s.sigma, s.rc, g)
    for p, q in zip(a, b):
        assert np.abs(p - q).max() < 1e-11 * np.abs(p).max()


# ---------------------------------------------------------------- input preparation


def test_random_sequential_addition_minimum_distances():
    """The random-start binary liquid: exact 80:20 composition, density 1.2,
    positions in [0, L), no pair (minimum image) closer than 0.8 sigma_ij,
    and the same arrays for the same seed."""
    s = inputs.binary_liquid_random(1500, seed=5)
    L = s.box[0]
    assert abs(s.n / L ** 3 - 1.2) < 1e-12
    assert int((s.types == 1).sum()) == 300
    assert np.all(s.x >= 0.0) and np.all(s.x < L)
    d = s.x[:, None, :] - s.x[None, :, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(axis=2))
    np.fill_diagonal(r, np.inf)
    dmin = 0.8 * s.sigma[s.types[:, None], s.types[None, :]]
    assert np.all(r >= dmin)
    s2 = inputs.binary_liquid_random(1500, seed=5)
    assert np.array_equal(s.x, s2.x) and np.array_equal(s.v, s2.v)


def test_equilibrate_rescales_to_temperature(oracle):
    """The equilibration run is velocity Verlet with the velocities rescaled
    after every step: the kinetic temperature (3n - 3 degrees of freedom) is
    the target after the run, the positions of a one-step run equal those
    of a plain one-step run (the rescaling follows the drift), and its
    velocities are the plain run's scaled by one common factor."""
    s = inputs.binary_liquid_random(600, seed=9)
    x1, v1 = oracle.equilibrate(s.x, s.v, s.types, s.box, s.eps, s.sigma, s.rc, s.mass, s.dt,
                                1, 0.5, s.skin)
    xp, vp, _, _ = oracle.md(s.x, s.v, s.types, s.box, s.eps, s.sigma, s.rc, s.mass, s.dt, 1,
                             skin=s.skin)
    assert np.array_equal(x1, xp)
    k = v1 / vp
    assert np.allclose(k, k.flat[0], rtol=1e-13, atol=0.0)
    for v in (v1, oracle.equilibrate(s.x, s.v, s.types, s.box, s.eps, s.sigma, s.rc, s.mass,
                                     s.dt, 40, 0.8, s.skin)[1]):
        temp = 2.0 * oracle.kinetic(v, s.types, s.mass) / (3 * s.n - 3)
        assert abs(temp - (0.5 if v is v1 else 0.8)) < 1e-12


def test_timing_build_agrees_with_parity_build(oracle):
    """The -O3 -march=native build used to time the oracle computes the same
    forces as the parity build (contraction may differ: within 1e-12)."""
    from oracle import ljref

    s = inputs.fcc_liquid(5)
    a = ljref.md(s.x, s.v, None, s.box, s.eps, s.sigma, s.rc, s.mass, s.dt, 10, skin=s.skin)
    b = ljref.md(s.x, s.v, None, s.box, s.eps, s.sigma, s.rc, s.mass, s.dt, 10, skin=s.skin,
                 timing=True)
    for p, q in zip(a[:3], b[:3]):
        assert np.abs(p - q).max() <= 1e-10 * max(np.abs(p).max(), 1.0)
