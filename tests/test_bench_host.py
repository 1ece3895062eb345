"""Host-side arithmetic of bench.py's report, on the CPU: the byte model and
roofline fraction of the dominant kernel, the path-level figure, the use of
the committed HBM counters, and the NVE drift statistics.  The numbers are
worked out by hand from the byte model (per atom: 4 for the row length, 4 per
list entry, 24 for x_i, 24 for f_i, 72 for the fused velocity-Verlet update;
per atom-step: integration 120, build (96 + 4 nbar) / 20)."""
import json
import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


class _Rows:
    """Stands in for a thermo tensor (bench reads .cpu().numpy())."""

    def __init__(self, a):
        self.a = np.asarray(a, dtype=np.float64)

    def cpu(self):
        return self

    def numpy(self):
        return self.a


def test_entry_bytes_model():
    force, integ, build = bench.entry_bytes_model(76.0)
    assert force == 4 + 4 * 76 + 24 + 24 == 356
    assert integ == 120
    assert build == pytest.approx((96 + 4 * 76) / 20.0)
    # a second type adds the 4-byte type of the home atom
    assert bench.entry_bytes_model(76.0, ntypes=2)[0] == 360


def test_roofline_by_hand():
    n, nbar, ms, launches = 2_048_000, 75.0, 0.2, 20
    phases = {"force": (ms * launches, launches), "build": (0.9, 1),
              "integrate": (0.0, 0), "other": (0.0, 0)}
    r = bench.roofline(n, nbar, phases, "tiled", 1, fused=True, ms_per_step=0.25)
    per_atom = 4 + 4 * nbar + 48 + 72  # 428
    assert r["algorithmic_bytes_per_atom"] == pytest.approx(per_atom)
    achieved = n * per_atom / (ms * 1e-3) / 1e9  # GB/s
    assert r["achieved"] == pytest.approx(achieved, abs=0.06)
    assert r["frac"] == pytest.approx(achieved / 8000.0, abs=1e-4)
    assert r["peak"] == 8000.0 and r["unit"] == "GB/s" and r["bound"] == "hbm"
    assert r["avg_launch_ms"] == pytest.approx(ms) and r["launches"] == launches
    # the bytes the tiled list stores: 2 per entry
    assert r["stored_list_bytes_per_atom"] == pytest.approx(4 + 2 * nbar + 48 + 72)
    # the whole step: force + integration + amortized build, over its time
    path_b = (4 + 4 * nbar + 48) + 120 + (96 + 4 * nbar) / 20
    assert r["path"]["bytes_per_atom_step"] == pytest.approx(path_b, abs=0.006)
    assert r["path"]["frac"] == pytest.approx(n * path_b / 0.25e-3 / 1e9 / 8000.0, abs=1e-4)
    # without the fused update the 72 bytes go
    r2 = bench.roofline(n, nbar, phases, "tiled", 1, fused=False, ms_per_step=0.25)
    assert r2["algorithmic_bytes_per_atom"] == pytest.approx(per_atom - 72)


def test_roofline_traffic_only_for_matching_counters():
    """traffic is the committed counters' HBM bytes when they were taken on
    the current kernel sources at this size and lane count, else null."""
    with open(bench.COUNTERS) as fh:
        c = json.load(fh)
    from paper_2508_13523_amd.profiling import gather_source_hash
    phases = {"force": (4.0, 20)}
    r = bench.roofline(c["atoms"], 75.0, phases, "tiled", 1, fused=True, ms_per_step=0.25)
    if c.get("kernel_source_sha256_16") == gather_source_hash():
        assert r["traffic"] == pytest.approx(c["hbm_bytes_per_launch"])
        # read and written bytes, each from its counter and the copy calibration
        assert c["hbm_bytes_per_launch"] == pytest.approx(
            c["hbm_read_bytes_per_launch"] + c["hbm_write_bytes_per_launch"])
        assert c["hbm_read_bytes_per_launch"] == pytest.approx(
            c["fetch_kib_per_dispatch"] * c["copy_bytes_per_fetch_kib"])
    else:
        assert r["traffic"] is None
    # another size or another lane count never takes them
    assert bench.roofline(c["atoms"] + 1, 75.0, phases, "tiled", 1, True, 0.25)["traffic"] is None
    assert bench.roofline(c["atoms"], 75.0, phases, "tiled", 2, True, 0.25)["traffic"] is None


def test_drift_stats_linear_energy():
    """E(t) = E0 + a t exactly: the slope is a per atom, the drift a t_end per
    atom, the largest excursion the same."""
    n, dt, a = 1000, 0.005, 3.0
    steps = np.arange(0, 1001, 100, dtype=np.float64)
    e = -5000.0 + a * steps * dt
    rows = np.zeros((len(steps), 9))
    rows[:, 0] = steps
    rows[:, 1] = e - 100.0  # potential
    rows[:, 2] = 100.0      # kinetic
    d = bench.drift_stats(_Rows(rows), n, dt)
    assert d["drift_slope_per_atom_per_tau"] == pytest.approx(a / n)
    assert d["energy_drift_per_atom"] == pytest.approx(a * 1000 * dt / n)
    assert d["max_energy_excursion_per_atom"] == pytest.approx(a * 1000 * dt / n)
    assert d["thermo_rows"] == len(steps) and d["steps"] == 1000


def test_drift_stats_returns_to_start():
    """An excursion that comes back: zero end drift, excursion its peak."""
    rows = np.zeros((3, 9))
    rows[:, 0] = [0, 10, 20]
    rows[:, 1] = [-10.0, -9.0, -10.0]
    d = bench.drift_stats(_Rows(rows), 10, 0.01)
    assert d["energy_drift_per_atom"] == 0.0
    assert d["max_energy_excursion_per_atom"] == pytest.approx(0.1)
    assert math.isclose(d["drift_slope_per_atom_per_tau"], 0.0, abs_tol=1e-12)
