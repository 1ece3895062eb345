#!/usr/bin/env python
"""Lennard-Jones MD benchmark on one MI355X: neighbor build + 12-6 force +
velocity Verlet at 2,048,000 atoms, FP64 and mixed precision, with the other
workloads of the method beside it.

Prints one JSON line.  `value` is FP64 throughput in millions of atom-steps
per second over K timed steps of the 2,048,000-atom FCC liquid (each step:
half kick + drift, a neighbor rebuild every 20 steps, the force evaluation,
half kick).  Inputs are synthetic and resident on the GPU before timing starts.

Every timed region is preceded by 100 ms (--settle-ms) of continuous GPU work
of its own leg (settle()).  The MD legs time their K steps without the
library's per-phase HIP events and then run K more steps with them, whose
per-phase GPU times (the force kernel's average launch, the roofline) they
report (run_md); the cold leg carries the events in its timed steps.

Legs (all on the GPU unless noted):
  drift        untimed 1,000-step FP64 and mixed runs at 2,048,000 atoms with
               thermo every 10 steps: NVE energy drift per atom and the mixed
               force error at identical positions (run before the timed leg)
  drift_long   the same FP64 and mixed runs over 10,000 steps (--drift-long-steps)
               with thermo every 100 steps
  fp64         the headline: set-up, untimed steps until the GPU has been busy
               for 100 ms (--settle-ms; whole rebuild intervals), W warm-up
               steps, then K timed steps
  cold         the same run with no settling, started after 0.5 s of idle GPU
               (its first milliseconds of load run slower: see settle())
  mixed, half  the same K steps in mixed precision, and with the half list
               (forces by atomic scatter)
  c1           4,000 atoms, 100 steps (eager and replayed from a HIP graph)
  c2           256,000 atoms, 1,000 steps, full-list gather vs half-list
               scatter, neighbor build timed apart from the force
  large        16,384,000 atoms, 1,000 steps, FP64 and mixed, each with its
               energy drift; mixed force error at identical positions
  adjoint      force-matching gradient rate, 32,000-atom binary liquid placed
               by random sequential addition and equilibrated 1,000 steps at
               T = 0.8 (velocity rescaling) with the library's own md_step
  batch        512 binary replicas: force-matching gradient and graph MD
  sweep        MD throughput from 4,000 to 8,388,608 atoms (full list FP64 and
               mixed, half list FP64) and the force gather's time at 1, 2, 4
               and 8 lanes per atom at each size
  cpu_baseline the oracle (serial C, -O3 -march=native build) on one host core
"""
import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Matom-steps/s LJ force+neigh @2M atoms: FP64 vs mixed; adjoint grads/s"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
COUNTERS = os.path.join(ROOT, "profiles", "force_gather_fp64_2048k_counters.json")
DEFAULT_VARIANTS = "drift,drift_long,fp64,cold,mixed,half,c1,c2,large,adjoint,batch,sweep"
SETTLE_MS = 100.0  # continuous GPU work before each timed region (see settle)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--ncell", type=int, default=80, help="FCC cells per side (80 -> 2,048,000 atoms)")
    ap.add_argument("--variants", default=DEFAULT_VARIANTS)
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--global-format", action="store_true",
                    help="build lists in the global (atom-index) format instead of tiled")
    ap.add_argument("--gather-lanes", type=int, default=0,
                    help="lanes per atom of the tiled full-list gather (1, 2, 4; 0: library default)")
    ap.add_argument("--drift-long-steps", type=int, default=10000,
                    help="steps of the long NVE runs (variant drift_long)")
    ap.add_argument("--settle-ms", type=float, default=SETTLE_MS,
                    help="continuous GPU work (ms) of each leg before its timed region")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference dispatch for counters)")
    return ap.parse_args()


# ------------------------------------------------------------------ MD runs


def settle(torch, work, ms, per_sync=10):
    """Calls `work` (GPU work of the leg about to be timed) until the GPU has
    been kept busy for `ms` milliseconds, synchronizing after every
    `per_sync` calls; returns the number of calls.  After an idle period the
    GPU runs these kernels 10-15% slower during its first 20-50 ms of
    continuous load (2,048,000 atoms: 0.352-0.356 ms per MD step cold,
    0.300 ms after 50-200 ms of force evaluations, on the same state), so a
    timed region of a few milliseconds right after set-up would measure that
    transient instead of the steady state of a continuous run."""
    if ms <= 0:
        return 0
    calls = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(per_sync):
            work()
        calls += per_sync
        torch.cuda.synchronize()
    return calls


def run_md(api, torch, s, params, steps, warmup, mixed=False, mode="full", rebuild=20,
           thermo_every=0, sort=True, global_format=False, settle_ms=None, phases="repeat"):
    """Set-up; untimed steps, in whole rebuild intervals, until the GPU has
    been busy for `settle_ms` (default SETTLE_MS; 0: none); `warmup` untimed
    steps; then `steps` timed steps.  Returns timing, per-phase GPU time (HIP
    events inside the library), the step counts and state.

    The library brackets each phase with two HIP events when asked to, and
    their packets between the kernels cost about 1-3% of a step at 2,048,000
    atoms, so with phases="repeat" the timed steps run without them and the
    next `steps` steps (the same trajectory, continued) run with them, for the
    per-phase times; with "inline" the timed steps themselves carry the
    events (the cold-start leg, whose kernels are timed in the transient
    itself); with None there are no phase times."""
    settle_ms = SETTLE_MS if settle_ms is None else settle_ms
    dev = torch.device("cuda")
    x = torch.tensor(s.x, device=dev)
    v = torch.tensor(s.v, device=dev)
    f = torch.zeros_like(x)
    cap = api.default_capacity(params, s.box, s.n)
    nl = api.NeighborList(s.n, cap, s.box, params, mode=mode, global_format=global_format)
    ws = api.workspace(s.n, s.box, params)
    api.md_step(x, v, f, None, s.box, params, nl, s.dt, 0, step0=0, rebuild_every=rebuild,
                setup=True, mixed=mixed, ws=ws, sort=sort)
    step = [0]

    def interval():
        api.md_step(x, v, f, None, s.box, params, nl, s.dt, rebuild, step0=step[0],
                    rebuild_every=rebuild, mixed=mixed, ws=ws, sort=sort)
        step[0] += rebuild

    settle(torch, interval, settle_ms, per_sync=1)
    settle_steps = step[0]
    api.md_step(x, v, f, None, s.box, params, nl, s.dt, warmup, step0=settle_steps,
                rebuild_every=rebuild, mixed=mixed, ws=ws, sort=sort)
    st = api.get_status(nl)
    if st[0]:
        raise RuntimeError(f"neighbor capacity {cap} exceeded in warm-up (need {st[1]})")
    first = settle_steps + warmup
    rows = api.thermo_rows(first, steps, thermo_every, False)
    thermo = torch.zeros((max(rows, 1), 9), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    api.profile_read()
    api.profile_enable(phases == "inline")
    t0 = time.perf_counter()
    api.md_step(x, v, f, None, s.box, params, nl, s.dt, steps, step0=first, rebuild_every=rebuild,
                thermo_every=thermo_every, mixed=mixed, ws=ws, thermo=thermo, sort=sort)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.profile_enable(False)
    ph = api.profile_read()
    phase_steps = [first, first + steps]
    if phases == "repeat":
        api.profile_enable(True)
        api.md_step(x, v, f, None, s.box, params, nl, s.dt, steps, step0=first + steps,
                    rebuild_every=rebuild, mixed=mixed, ws=ws, sort=sort)
        torch.cuda.synchronize()
        api.profile_enable(False)
        ph = api.profile_read()
        phase_steps = [first + steps, first + 2 * steps]
    st = api.get_status(nl)
    if st[0]:
        raise RuntimeError(f"neighbor capacity {cap} exceeded (need {st[1]})")
    nbar = float(nl.numneigh[: s.n].to(torch.float64).mean().item())
    return dict(seconds=t1 - t0, phases=ph, status=st.tolist(), nbar=nbar, x=x, v=v, f=f,
                nl=nl, thermo=thermo[:rows], ws=ws, format=nl.format, tile=list(nl.tile),
                settle_steps=settle_steps, first_timed_step=first, phase_steps=phase_steps)


def drift_stats(thermo, n, dt):
    """NVE energy drift of thermo rows [g, E_pot, KE, ...]: |E(end) - E(0)| / N,
    the largest |E(t) - E(0)| / N, and the least-squares slope of
    (E(t) - E(0)) / N per unit time (tau)."""
    th = thermo.cpu().numpy()
    e = th[:, 1] + th[:, 2]
    t = th[:, 0] * dt
    de = (e - e[0]) / n
    slope = float(np.polyfit(t, de, 1)[0]) if len(t) >= 2 else 0.0
    return {"energy_drift_per_atom": float(abs(de[-1])),
            "max_energy_excursion_per_atom": float(np.abs(de).max()),
            "drift_slope_per_atom_per_tau": slope,
            "thermo_rows": int(len(t)), "steps": int(th[-1, 0] - th[0, 0])}


def force_error(api, s, params, x, nl, ws):
    """Mixed-precision force error at identical positions: max |dF| / max |F|
    (componentwise) and max_i |dF_i| / F_rms, against the FP64 path."""
    f64, _ = api.lj_forces(x, None, s.box, params, nl, ws=ws)
    f32, _ = api.lj_forces(x, None, s.box, params, nl, mixed=True, ws=ws)
    d = (f32 - f64).abs()
    return {"max_abs_dF_over_max_abs_F": float(d.max() / f64.abs().max()),
            "max_norm_dF_over_F_rms": float(d.norm(dim=1).max() /
                                            f64.norm(dim=1).pow(2).mean().sqrt())}


def drift_runs(api, torch, s, params, steps=1000, thermo_every=10):
    """Untimed NVE runs of `steps` steps (rebuild every 20, atoms sorted), FP64
    and mixed, from the same start: each run's drift, and the mixed force
    error at the mixed run's final positions."""
    out = {}
    for name, mixed in (("fp64", False), ("mixed", True)):
        r = run_md(api, torch, s, params, steps, 0, mixed=mixed, thermo_every=thermo_every,
                   settle_ms=0, phases=None)
        out[name] = drift_stats(r["thermo"], s.n, s.dt)
        out[name]["seconds"] = round(r["seconds"], 4)
        if mixed:
            out[name].update(force_error(api, s, params, r["x"], r["nl"], r["ws"]))
        del r
        torch.cuda.empty_cache()
    return out


def entry_bytes_model(nbar, ntypes=1):
    """Algorithmic bytes per atom and step of the full-list path: force
    4 (row length) + 4 nbar (4-byte list entries) + 24 (x_i) + 24 (f_i)
    (+ 4 for the type when several), integration 120 (read x, v, f; write x, v),
    build (96 + 4 nbar) / 20 (amortized over the 20-step rebuild interval)."""
    force = 4.0 + 4.0 * nbar + 24.0 + 24.0 + (4.0 if ntypes > 1 else 0.0)
    return force, 120.0, (96.0 + 4.0 * nbar) / 20.0


def roofline(N, nbar, phases, fmt, lanes, fused, ms_per_step):
    """Roofline of the dominant kernel (the FP64 full-list gather).  Algorithmic
    bytes per launch = N x (4 + 4 nbar + 24 + 24) (row length, 4-byte list
    entries, x_i, f_i); in the MD step with a tiled full list the kernel also
    applies the velocity-Verlet update, which adds 72 bytes per atom (read and
    write v_i, write the drifted x_i).  The bytes the tiled list actually
    stores per entry (2) are reported apart.  `path` is the whole step
    (force + integration + amortized build) against its mean time."""
    ms, launches = phases["force"]
    avg_ms = ms / max(launches, 1)
    force_b, integ_b, build_b = entry_bytes_model(nbar)
    per_atom = force_b + (72.0 if fused else 0.0)
    bytes_per_launch = N * per_atom
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    entry = 2.0 if fmt == "tiled" else 4.0
    moved = 4.0 + entry * nbar + 48.0 + (72.0 if fused else 0.0)
    traffic = None
    try:
        with open(COUNTERS) as fh:
            c = json.load(fh)
        from paper_2508_13523_amd.profiling import gather_kernel, gather_source_hash
        if (c.get("kernel_source_sha256_16") == gather_source_hash() and c.get("atoms") == N
                and c.get("kernel") == gather_kernel(lanes)):
            traffic = c["hbm_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        traffic = None
    path_b = force_b + integ_b + build_b
    path_gbs = N * path_b / (ms_per_step * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": (f"k_force_tile_gather<1,false,false,{lanes},false>" if fmt == "tiled" else
                       "k_force_gather<1,false,false>") + " (FP64 full-list gather" +
                      (", fused velocity-Verlet update)" if fused else ")"),
            "algorithmic_bytes_per_atom": round(per_atom, 2),
            "byte_model": "4 + 4 nbar + 24 + 24 per atom (4-byte entries)"
                          + (" + 72 fused update" if fused else ""),
            "stored_list_bytes_per_atom": round(moved, 2),
            "avg_launch_ms": round(avg_ms, 5), "launches": launches,
            "algorithmic_bytes_per_launch": int(bytes_per_launch),
            "mean_neighbors": round(nbar, 3),
            "path": {"bytes_per_atom_step": round(path_b, 2),
                     "terms": {"force": round(force_b, 2), "integrate": integ_b,
                               "build_amortized": round(build_b, 2)},
                     "achieved": round(path_gbs, 1),
                     "frac": round(path_gbs / HBM_PEAK_GBS, 4)}}


def md_leg(api, torch, s, params, K, W, mixed=False, mode="full", global_format=False,
           settle_ms=None, phases="repeat"):
    r = run_md(api, torch, s, params, K, W, mixed=mixed, mode=mode, global_format=global_format,
               settle_ms=settle_ms, phases=phases)
    out = {"value": round(s.n * K / r["seconds"] / 1e6, 2),
           "ms_per_step": round(r["seconds"] / K * 1e3, 4),
           "force_kernel_ms": round(r["phases"]["force"][0] / max(r["phases"]["force"][1], 1), 5),
           "mean_neighbors": round(r["nbar"], 3)}
    return out, r


def phase_split(r, steps):
    """Per-phase times of a run: force per launch, build per rebuild, and the
    per-step share of each phase."""
    ph = r["phases"]
    out = {k: round(v[0] / steps, 5) for k, v in ph.items()}
    fb = ph.get("build", (0.0, 0))
    ff = ph.get("force", (0.0, 0))
    return {"ms_per_step_by_phase": out,
            "build_ms_per_rebuild": round(fb[0] / max(fb[1], 1), 5),
            "rebuilds": fb[1],
            "force_ms_per_launch": round(ff[0] / max(ff[1], 1), 5)}


def graph_md_rate(api, torch, s, params, steps=200, reps=3):
    """FP64 MD throughput with `steps` steps (rebuild every 20, atoms sorted)
    captured once in a HIP graph and replayed: the step's kernels without
    the host's launch overhead, which bounds small systems."""
    dev = torch.device("cuda")
    x = torch.tensor(s.x, device=dev)
    v = torch.tensor(s.v, device=dev)
    f = torch.zeros_like(x)
    cap = api.default_capacity(params, s.box, s.n)
    nl = api.NeighborList(s.n, cap, s.box, params)
    ws = api.workspace(s.n, s.box, params)
    api.md_step(x, v, f, None, s.box, params, nl, s.dt, 20, step0=0, setup=True, ws=ws,
                sort=True)
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            api.md_step(x, v, f, None, s.box, params, nl, s.dt, steps, step0=20, ws=ws,
                        sort=True)
    torch.cuda.current_stream().wait_stream(st)
    g.replay()
    settle(torch, g.replay, SETTLE_MS, per_sync=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / (reps * steps)
    st_ = api.get_status(nl)
    if st_[0]:
        raise RuntimeError(f"neighbor capacity {cap} exceeded (need {st_[1]})")
    return {"Matom_steps_per_s": round(s.n / dt / 1e6, 2), "us_per_step": round(dt * 1e6, 2),
            "steps": steps}


def c1_leg(api, torch, inputs):
    """4,000 atoms (10^3 FCC cells), 100 steps with rebuild every 20, FP64
    full list: eager library calls, and the 100 steps replayed from a HIP
    graph (small systems are bound by the host's launches)."""
    s = inputs.fcc_liquid(10)
    p = api.LJParams.from_system(s)
    r = run_md(api, torch, s, p, 100, 0)
    out = {"atoms": s.n, "steps": 100,
           "eager_Matom_steps_per_s": round(s.n * 100 / r["seconds"] / 1e6, 2),
           "eager_ms_per_step": round(r["seconds"] / 100 * 1e3, 4)}
    out.update(phase_split(r, 100))
    out["graph"] = graph_md_rate(api, torch, s, p, steps=100, reps=5)
    return out


def c2_leg(api, torch, inputs, steps=1000):
    """256,000 atoms (40^3 FCC cells), `steps` steps with rebuild every 20:
    the full-list gather and the half-list scatter, each with its neighbor
    build timed apart from the force."""
    s = inputs.fcc_liquid(40)
    p = api.LJParams.from_system(s)
    out = {"atoms": s.n, "steps": steps}
    for name, mode in (("gather_full", "full"), ("scatter_half", "half")):
        r = run_md(api, torch, s, p, steps, 20, mode=mode)
        row = {"Matom_steps_per_s": round(s.n * steps / r["seconds"] / 1e6, 2),
               "ms_per_step": round(r["seconds"] / steps * 1e3, 4),
               "mean_neighbors": round(r["nbar"], 3)}
        row.update(phase_split(r, steps))
        out[name] = row
        del r
    out["gather_over_scatter"] = round(out["gather_full"]["Matom_steps_per_s"] /
                                       out["scatter_half"]["Matom_steps_per_s"], 3)
    return out


def large_leg(api, torch, inputs, steps=1000, warmup=20, ncell=160):
    """16,384,000 atoms (160^3 FCC cells), FP64 and mixed precision, each
    `steps` timed steps with rebuild every 20 and thermo every 100: throughput,
    each run's energy drift, and the mixed force error at identical
    positions."""
    s16 = inputs.fcc_liquid(ncell)
    p16 = api.LJParams.from_system(s16)
    n = s16.n
    res = {"atoms": n, "steps": steps}
    for name, mixed in (("fp64", False), ("mixed", True)):
        r = run_md(api, torch, s16, p16, steps, warmup, mixed=mixed, thermo_every=100)
        row = {"value": round(n * steps / r["seconds"] / 1e6, 2),
               "ms_per_step": round(r["seconds"] / steps * 1e3, 4),
               "force_kernel_ms": round(r["phases"]["force"][0] /
                                        max(r["phases"]["force"][1], 1), 5)}
        row.update(drift_stats(r["thermo"], n, s16.dt))
        if mixed:
            row.update(force_error(api, s16, p16, r["x"], r["nl"], r["ws"]))
        res[name] = row
        del r
        torch.cuda.empty_cache()
    res["mixed"]["speedup_vs_fp64"] = round(res["mixed"]["value"] / res["fp64"]["value"], 3)
    return res


# ------------------------------------------------------------------ adjoint


def equilibrated_binary(api, torch, inputs, n=32000, seed=3, steps=1000, temperature=0.8):
    """The force-matching input: 80:20 binary liquid at density 1.2 placed by
    random sequential addition (minimum distance 0.8 sigma_ij), then `steps`
    velocity-Verlet steps (dt 0.005, list rebuilt every 20 steps) on the GPU
    with the library's md_step, the velocities rescaled to T = 0.8 after each
    step.  Returns (system, x, v, types) with x, v, types on the GPU."""
    s = inputs.binary_liquid_random(n, seed=seed)
    params = api.LJParams.from_system(s)
    dev = torch.device("cuda")
    x = torch.tensor(s.x, device=dev)
    v = torch.tensor(s.v, device=dev)
    t = torch.tensor(s.types, device=dev, dtype=torch.int32)
    f = torch.zeros_like(x)
    nl = api.NeighborList(s.n, api.default_capacity(params, s.box, s.n), s.box, params)
    ws = api.workspace(s.n, s.box, params)
    target = 0.5 * (3 * n - 3) * temperature
    api.md_step(x, v, f, t, s.box, params, nl, s.dt, 0, setup=True, ws=ws)
    for k in range(steps):
        api.md_step(x, v, f, t, s.box, params, nl, s.dt, 1, step0=k, rebuild_every=20, ws=ws)
        ke = 0.5 * (v * v).sum()  # unit masses
        v.mul_(torch.sqrt(target / ke))
    st = api.get_status(nl)
    if st[0] or st[3]:
        raise RuntimeError(f"equilibration failed: status {st}")
    return s, x, v, t


def adjoint_rate(api, torch, inputs, evals=200):
    """Force-matching gradient evaluations per second on the 32,000-atom
    binary liquid (equilibrated as in equilibrated_binary): forward F, loss
    gradient g = 2 (F - F_t) / N, adjoint to x, eps, sigma.  Timed eagerly
    (one library call per kernel) and with the whole evaluation captured once
    in a HIP graph and replayed; every replay's gradients are checked against
    the eager ones; grads_per_s is the faster of the two."""
    t_prep = time.perf_counter()
    s, x, _, t = equilibrated_binary(api, torch, inputs)
    t_prep = time.perf_counter() - t_prep
    params = api.LJParams.from_system(s)
    dev = torch.device("cuda")
    nl = api.build_list(x, t, s.box, params)
    # the atoms put into cell order once, untimed (the order the MD keeps by
    # sorting at each rebuild); the list is rebuilt with it
    api.md_step(x, torch.zeros_like(x), torch.empty_like(x), t, s.box, params, nl, s.dt, 0,
                setup=True, sort=True)
    e_t, s_t = inputs.perturbed_params(s.eps, s.sigma, seed=4)
    ft, _ = api.lj_forces(x, t, s.box, api.LJParams(e_t, s_t, s.rc, s.skin), nl)
    ws = api.workspace(s.n, s.box, params)
    f = torch.empty_like(x)
    g = torch.empty_like(x)

    gxo = torch.empty_like(x)

    def grad():
        return api.fm_grad(x, t, s.box, params, nl, ft, ws=ws, gx=gxo)

    def composed():
        api.lj_forces(x, t, s.box, params, nl, f=f, ws=ws)
        torch.sub(f, ft, out=g).mul_(2.0 / s.n)
        return api.lj_backward(x, t, s.box, params, nl, g, ws=ws)

    for _ in range(5):
        ref = grad()
    ref = [r.clone() for r in ref]
    comp = composed()
    same_as_composed = all(torch.equal(a, b) for a, b in zip(ref, comp))
    settle(torch, grad, SETTLE_MS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(evals):
        composed()
    torch.cuda.synchronize()
    dt_composed = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(evals):
        grad()
    torch.cuda.synchronize()
    dt_eager = time.perf_counter() - t0

    graph = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(graph, stream=st):
            out = grad()
    torch.cuda.current_stream().wait_stream(st)
    mismatch = 0
    for _ in range(3):  # replays checked against the eager result, eager work between
        graph.replay()
        torch.cuda.synchronize()
        mismatch += sum(int(not torch.equal(a, b)) for a, b in zip(out, ref))
        grad()
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(evals):
        graph.replay()
    torch.cuda.synchronize()
    dt_graph = time.perf_counter() - t0
    mismatch += sum(int(not torch.equal(a, b)) for a, b in zip(out, ref))
    best = min(dt_eager, dt_graph)
    return {"grads_per_s": round(evals / best, 1), "atoms": s.n, "evals": evals,
            "ms_per_grad": round(best / evals * 1e3, 4),
            "eager_grads_per_s": round(evals / dt_eager, 1),
            "graph_grads_per_s": round(evals / dt_graph, 1),
            "graph_replays_equal_eager": mismatch == 0,
            "composed_ms_per_grad": round(dt_composed / evals * 1e3, 4),
            "fused_equals_composed": same_as_composed,
            "input_preparation_s": round(t_prep, 2),
            "workload": "binary LJ 80:20, 32,000 atoms, rho 1.2, random sequential addition "
                        "then 1,000 steps at T 0.8 (velocity rescaling); FP64 forward + "
                        "adjoint to positions and the 2x2 eps/sigma tables in one ljmd_fm_grad "
                        "call (the gather writes the loss gradient); atoms in cell order "
                        "(sorted once before timing); the faster of eager calls and one HIP "
                        "graph per evaluation; composed_ms_per_grad: forces, torch g, adjoint"}


def equilibrate_batch(B, torch, bt, prm, nl, ws, x, v, t, sizes, steps=1000, temperature=0.8,
                      dt=0.005):
    """`steps` velocity-Verlet steps of every system (FP64, list rebuilt every
    20 steps, atoms sorted at each rebuild), each system's velocities rescaled
    to `temperature` (3 N_r - 3 degrees of freedom, unit masses) after every
    step from the kinetic energy in its thermo row."""
    dev = x.device
    n_r = torch.tensor(sizes, dtype=torch.float64, device=dev)
    target = 0.5 * (3.0 * n_r - 3.0) * temperature
    counts = torch.tensor(sizes, dtype=torch.int64, device=dev)
    f = torch.zeros_like(x)
    B.md_step(x, v, f, t, bt, prm, nl, dt, 0, setup=True, sort=True, ws=ws)
    for k in range(steps):
        rows = B.md_step(x, v, f, t, bt, prm, nl, dt, 1, step0=k, rebuild_every=20,
                         thermo_every=1, sort=True, ws=ws)
        ke = rows[0, :, 2]
        v.mul_(torch.repeat_interleave(torch.sqrt(target / ke), counts)[:, None])
    st = B.get_status(nl)
    if st[0] or st[3]:
        raise RuntimeError(f"batch equilibration failed: status {st}")


def batch_rates(api, torch, inputs, replicas=512, iters=20, md_steps=100, equil_steps=1000):
    """Batched replicas: R binary-liquid systems with atom counts uniform on
    [500, 8000] (seed 6), system r prepared with seed 1000 + r.
      - force matching: mixed-precision forward + FP64 adjoint of all systems
        per iteration (one launch per kernel), against the same work done
        system by system with the single-system FP64 calls;
      - MD: the batch velocity-Verlet step (rebuild every 20) captured once in
        a HIP graph and replayed."""
    from paper_2508_13523_amd import batch as B

    sizes = inputs.replica_sizes(replicas, seed=6)
    rb = inputs.replica_batch(sizes, seed_base=1000)
    dev = torch.device("cuda")
    bt = B.Batch(rb["offsets"], rb["boxes"])
    prm = api.LJParams(rb["eps"], rb["sigma"], rb["rc"], rb["skin"], rb["mass"])
    x = torch.tensor(rb["x"], device=dev)
    t = torch.tensor(rb["types"], device=dev, dtype=torch.int32)
    v = torch.tensor(rb["v"], device=dev)
    nl = B.build_list(x, t, bt, prm)
    ws = B.workspace(bt, prm)
    # untimed: every system equilibrated 1,000 steps at T = 0.8 (velocity
    # rescaling per system after each step, atoms kept in cell order by
    # sorting at each rebuild), then the list rebuilt for the final positions
    t_eq = time.perf_counter()
    equilibrate_batch(B, torch, bt, prm, nl, ws, x, v, t, sizes, steps=equil_steps)
    t_eq = time.perf_counter() - t_eq
    B.md_step(x, v, torch.empty_like(x), t, bt, prm, nl, 0.005, 0, setup=True, mixed=True,
              sort=True, ws=ws)
    # tile target, lanes per atom and persistence tuned on this batch (the
    # list is left built for the chosen tiling), then the atoms re-sorted and
    # the list rebuilt as the MD does
    tuning = B.autotune(x, t, bt, prm, nl, mixed=True, tiles=True)
    ws = B.workspace(bt, prm)
    B.md_step(x, v, torch.empty_like(x), t, bt, prm, nl, 0.005, 0, setup=True, mixed=True,
              sort=True, ws=ws)
    x0, v0 = x.clone(), v.clone()
    e_t, s_t = inputs.perturbed_params(rb["eps"], rb["sigma"], seed=4)
    prm_t = api.LJParams(e_t, s_t, rb["rc"], rb["skin"], rb["mass"])
    ft, _ = B.lj_forces(x, t, bt, prm_t, nl, ws=ws)
    # loss = sum_r (1/N_r) sum_i |F_i - F_t,i|^2  ->  g_i = 2 (F_i - F_t,i) / N_r
    scale = torch.tensor(np.repeat(2.0 / sizes.astype(np.float64), sizes)[:, None], device=dev)
    f = torch.empty_like(x)
    gxo = torch.empty_like(x)

    def batched():
        return B.fm_grad(x, t, bt, prm, nl, ft, mixed=True, ws=ws, gx=gxo)

    def composed():
        B.lj_forces(x, t, bt, prm, nl, mixed=True, f=f, ws=ws)
        g = (f - ft).mul_(scale)
        return B.lj_backward(x, t, bt, prm, nl, g, ws=ws)

    ref = [r.clone() for r in batched()]
    same_as_composed = all(torch.equal(a, b) for a, b in zip(ref, composed()))
    settle(torch, batched, SETTLE_MS, per_sync=5)
    for _ in range(3):
        composed()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        composed()
    torch.cuda.synchronize()
    t_composed = (time.perf_counter() - t0) / iters
    for _ in range(3):
        batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        batched()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / iters

    # the same gradients system by system (single-system FP64 calls)
    singles = []
    for r, sysr in enumerate(rb["systems"]):
        sl = bt.system(r)
        xr = x[sl].contiguous()
        tr = t[sl].contiguous()
        p1 = api.LJParams.from_system(sysr)
        nl1 = api.build_list(xr, tr, sysr.box, p1)
        singles.append((xr, tr, sysr.box, p1, nl1, api.workspace(sysr.n, sysr.box, p1),
                        ft[sl].contiguous(), 2.0 / sysr.n))

    def sequential():
        for xr, tr, box, p1, nl1, w1, ftr, sc in singles:
            fr, _ = api.lj_forces(xr, tr, box, p1, nl1, ws=w1)
            api.lj_backward(xr, tr, box, p1, nl1, (fr - ftr).mul_(sc), ws=w1)

    sequential()
    torch.cuda.synchronize()
    seq_iters = max(2, iters // 5)
    t0 = time.perf_counter()
    for _ in range(seq_iters):
        sequential()
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / seq_iters

    # MD: graph-captured batch step, atoms re-sorted into cell order at every
    # rebuild, on a tiling tuned for the MD step (force + build / 20)
    x.copy_(x0)
    v.copy_(v0)
    fm = torch.zeros_like(x)
    btm = B.Batch(rb["offsets"], rb["boxes"])
    nlm = B.neighbor_list(btm, prm, nl.cap)
    wsm = B.workspace(btm, prm)
    B.md_step(x, v, fm, t, btm, prm, nlm, 0.005, 0, setup=True, mixed=True, sort=True, ws=wsm)
    tuning_md = B.autotune(x, t, btm, prm, nlm, mixed=True, tiles=True, for_md=True)
    wsm = B.workspace(btm, prm)
    B.md_step(x, v, fm, t, btm, prm, nlm, 0.005, 0, setup=True, mixed=True, sort=True, ws=wsm)
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            B.md_step(x, v, fm, t, btm, prm, nlm, 0.005, md_steps, step0=0, rebuild_every=20,
                      mixed=True, sort=True, ws=wsm)
    torch.cuda.current_stream().wait_stream(st)
    g.replay()
    settle(torch, g.replay, SETTLE_MS, per_sync=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    t_md = (time.perf_counter() - t0) / (reps * md_steps)
    stat = B.get_status(nlm)
    n = bt.n
    return {"replicas": replicas, "atoms": n, "sizes": [int(sizes.min()), int(sizes.max())],
            "tuning": {"lanes_per_atom": tuning[0], "block": tuning[1],
                       "persistent": tuning[2], "tile_atoms": tuning[3]},
            "tuning_md": {"lanes_per_atom": tuning_md[0], "block": tuning_md[1],
                          "persistent": tuning_md[2], "tile_atoms": tuning_md[3]},
            "replica_grads_per_s": round(replicas / t_batch, 1),
            "atom_grads_per_s": round(n / t_batch, 1),
            "ms_per_batch_grad": round(t_batch * 1e3, 4),
            "composed_ms_per_batch_grad": round(t_composed * 1e3, 4),
            "fused_equals_composed": same_as_composed,
            "sequential_fp64_ms_per_batch_grad": round(t_seq * 1e3, 4),
            "speedup_vs_sequential": round(t_seq / t_batch, 2),
            "md_graph_matom_steps_per_s": round(n / t_md / 1e6, 2),
            "md_graph_ms_per_step": round(t_md * 1e3, 4),
            "md_status_overflow": int(stat[0]),
            "equilibration_steps": equil_steps,
            "equilibration_s": round(t_eq, 2),
            "workload": "512 binary LJ 80:20 replicas, N_r uniform on [500, 8000], rho 1.2, "
                        "T 0.8, jittered random grid sites equilibrated 1,000 steps at T 0.8 "
                        "(velocity rescaling per system); mixed forward + FP64 adjoint per "
                        "force-matching gradient in one ljmd_batch_fm_grad call (composed: "
                        "forces, torch g, adjoint); MD with rebuild every 20 captured in one HIP "
                        "graph; atoms in cell order (sorted once before the gradients, at every "
                        "rebuild in the MD)"}


# ------------------------------------------------------------------ sweep


def gather_lane_times(api, torch, s, p, lanes_set=(1, 2, 4, 8), reps=20):
    """Mean time of one FP64 full-list force evaluation (tiled gather, no
    energy/virial) with 1, 2, 4 and 8 lanes sharing each atom's row (the
    paper's neighbor threading), on one list built from the sorted atoms."""
    dev = torch.device("cuda")
    x = torch.tensor(s.x, device=dev)
    v = torch.tensor(s.v, device=dev)
    f = torch.zeros_like(x)
    nl = api.NeighborList(s.n, api.default_capacity(p, s.box, s.n), s.box, p)
    ws = api.workspace(s.n, s.box, p)
    api.md_step(x, v, f, None, s.box, p, nl, s.dt, 0, setup=True, sort=True, ws=ws)
    out = {}
    settle(torch, lambda: api.lj_forces(x, None, s.box, p, nl, f=f, ws=ws), SETTLE_MS)
    prev = api.get_gather_lanes()
    try:
        for lanes in lanes_set:
            api.set_gather_lanes(lanes)
            for _ in range(3):
                api.lj_forces(x, None, s.box, p, nl, f=f, ws=ws)
            torch.cuda.synchronize()
            api.profile_read()
            api.profile_enable(True)
            for _ in range(reps):
                api.lj_forces(x, None, s.box, p, nl, f=f, ws=ws)
            torch.cuda.synchronize()
            api.profile_enable(False)
            ms, cnt = api.profile_read()["force"]
            out[str(lanes)] = round(ms / max(cnt, 1) * 1e3, 2)
    finally:
        api.set_gather_lanes(prev)
    auto = api.nl_gather_lanes(nl, s.box, p)
    return {"force_us_by_lanes_per_atom": out, "library_choice": auto}


def sweep_rates(api, torch, inputs, cells=(10, 20, 32, 50, 80, 128)):
    """Saturation sweep: MD throughput (rebuild every 20, atoms sorted into
    cell order) from 4,000 to 8,388,608 atoms: full list in FP64 and mixed,
    and the FP64 half list (Newton's third law, forces by scatter), so that
    the two list styles can be compared at every size; about 40 ms of timed
    full-list steps per size (100 to 2,000 steps; the half list runs as many
    steps).  Beside them, the force gather's time at 1, 2, 4 and 8 lanes per
    atom (the neighbor-threading comparison) and, up to 256,000 atoms, the
    FP64 MD replayed from a HIP graph."""
    rows = []
    for nc in cells:
        s = inputs.fcc_liquid(nc)
        p = api.LJParams.from_system(s)
        row = {"fcc_cells": nc, "atoms": s.n}
        steps = min(2000, max(100, int(4e-2 / (s.n * 1.6e-10)) // 20 * 20))
        for name, mixed, mode in (("fp64", False, "full"), ("mixed", True, "full"),
                                  ("half_fp64", False, "half")):
            r = run_md(api, torch, s, p, steps, 20, mixed=mixed, mode=mode)
            fph = r["phases"].get("force", (0.0, 0))
            row[name] = {"Matom_steps_per_s": round(s.n * steps / r["seconds"] / 1e6, 2),
                         "us_per_step": round(r["seconds"] / steps * 1e6, 2),
                         "force_phase_us": round(fph[0] / max(fph[1], 1) * 1e3, 2),
                         "steps": steps}
            del r
            torch.cuda.empty_cache()
        row["gather_lanes"] = gather_lane_times(api, torch, s, p)
        if s.n <= 300_000:
            row["fp64_graph"] = graph_md_rate(api, torch, s, p)
        log(f"sweep {nc}^3 cells, {s.n} atoms: {row['fp64']['Matom_steps_per_s']} / "
            f"{row['mixed']['Matom_steps_per_s']} / {row['half_fp64']['Matom_steps_per_s']} "
            f"Matom-steps/s (FP64 / mixed / FP64 half list); gather us by lanes "
            f"{row['gather_lanes']['force_us_by_lanes_per_atom']}")
        rows.append(row)
        torch.cuda.empty_cache()
    return rows


# ------------------------------------------------------------------ CPU baseline


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(s, steps):
    """The oracle (serial C, FP64, Verlet list rebuilt every 20 steps), built
    -O3 -march=native for timing, on one host core: the 2,048,000-atom system,
    time of (set-up + `steps` steps) minus time of set-up alone = one list
    build plus `steps` force/integration steps; and the whole 4,000-atom,
    100-step run."""
    from oracle import ljref
    from paper_2508_13523_amd import inputs

    ljref.lib(timing=True)
    t0 = time.perf_counter()
    ljref.md(s.x, s.v, None, s.box, s.eps, s.sigma, s.rc, s.mass, s.dt, 0, rebuild_every=20,
             skin=s.skin, timing=True)
    t1 = time.perf_counter()
    ljref.md(s.x, s.v, None, s.box, s.eps, s.sigma, s.rc, s.mass, s.dt, steps, rebuild_every=20,
             skin=s.skin, timing=True)
    t2 = time.perf_counter()
    per = (t2 - t1) - (t1 - t0)
    c1 = inputs.fcc_liquid(10)
    t3 = time.perf_counter()
    ljref.md(c1.x, c1.v, None, c1.box, c1.eps, c1.sigma, c1.rc, c1.mass, c1.dt, 100,
             rebuild_every=20, skin=c1.skin, timing=True)
    t4 = time.perf_counter()
    return {"value": round(s.n * steps / per / 1e6, 4), "unit": "Matom-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{s.n} atoms, {steps} steps incl. one list rebuild (set-up timed "
                      f"separately and subtracted); {t2 - t0:.1f} s of CPU work",
            "build": "gcc -O3 -march=native (oracle/build.py build_timing), one thread",
            "cpu_model": cpu_model(), "host_logical_cpus": os.cpu_count(),
            "c1_4000_atoms_100_steps_Matom_steps_per_s": round(c1.n * 100 / (t4 - t3) / 1e6, 4)}


# ------------------------------------------------------------------ main


def main():
    global SETTLE_MS
    args = parse()
    SETTLE_MS = args.settle_ms
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(replicas and spatial decomposition shard across GPUs by design, but only "
              "the single-GPU kernels are implemented). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2508_13523_amd import api, inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    variants = set(args.variants.split(","))
    api.set_gather_lanes(args.gather_lanes)
    s = inputs.fcc_liquid(args.ncell)
    params = api.LJParams.from_system(s)
    N, K, W = s.n, args.steps, args.warmup

    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    out = {"metric": METRIC, "value": None, "unit": "Matom-steps/s", "n_gpus": 1, "steps": K,
           "warmup": W, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"LJ 12-6 FCC liquid, {N} atoms ({args.ncell}^3 FCC cells), "
                                  "rho 0.8442, T 1.44, eps=sigma=1, rc 2.5, skin 0.3, full list "
                                  "gather, velocity Verlet dt 0.005, rebuild every 20 with atoms "
                                  "sorted into cell order",
                      "atoms": N, "rebuild_every": 20, "list": "full"}}

    if "drift" in variants:
        log("drift: 1,000-step FP64 and mixed runs at the benchmark size")
        out["drift_1000_steps"] = drift_runs(api, torch, s, params)
    if "drift_long" in variants:
        log(f"drift_long: {args.drift_long_steps}-step FP64 and mixed runs, thermo every 100")
        out["drift_long"] = drift_runs(api, torch, s, params, steps=args.drift_long_steps,
                                       thermo_every=100)
    fp64 = None
    if "fp64" in variants:
        log(f"fp64: {W} warm-up + {K} timed steps")
        fp64 = run_md(api, torch, s, params, K, W, global_format=args.global_format)
        out["value"] = round(N * K / fp64["seconds"] / 1e6, 2)
        out["ms_per_step"] = round(fp64["seconds"] / K * 1e3, 4)
        out["phases_ms_per_step"] = {k: round(v[0] / K, 5) for k, v in fp64["phases"].items()}
        lanes = api.nl_gather_lanes(fp64["nl"], s.box, params)
        out["roofline"] = roofline(N, fp64["nbar"], fp64["phases"], fp64["format"], lanes,
                                   fused=fp64["format"] == "tiled",
                                   ms_per_step=out["ms_per_step"])
        out["config"]["list_format"] = fp64["format"]
        out["config"]["gather_lanes_per_atom"] = lanes
        out["config"]["tile_cells"] = fp64["tile"]
        out["dangerous_builds_flagged"] = bool(fp64["status"][2])
        out["settle"] = {"ms": SETTLE_MS, "md_steps": fp64["settle_steps"],
                         "timed_steps": [fp64["first_timed_step"], fp64["first_timed_step"] + K],
                         "phase_event_steps": fp64["phase_steps"]}
        if "drift" in variants:
            out["fp64_energy_drift_per_atom"] = out["drift_1000_steps"]["fp64"][
                "energy_drift_per_atom"]
        del fp64["x"], fp64["v"], fp64["f"], fp64["nl"]
        torch.cuda.empty_cache()
    if "cold" in variants:
        log(f"cold: 0.5 s idle, then {W} warm-up + {K} timed steps with no settling")
        time.sleep(0.5)
        r, cold = md_leg(api, torch, s, params, K, W, global_format=args.global_format,
                         settle_ms=0, phases="inline")
        r["idle_s_before"] = 0.5
        r["timed_steps"] = [cold["first_timed_step"], cold["first_timed_step"] + K]
        out["cold_start"] = r
        del cold
        torch.cuda.empty_cache()
    if "mixed" in variants:
        log(f"mixed: {W} warm-up + {K} timed steps")
        r, mx = md_leg(api, torch, s, params, K, W, mixed=True, global_format=args.global_format)
        if "drift" in variants:
            d = out["drift_1000_steps"]["mixed"]
            r["energy_drift_per_atom"] = d["energy_drift_per_atom"]
            r["max_abs_dF_over_max_abs_F"] = d["max_abs_dF_over_max_abs_F"]
            r["max_norm_dF_over_F_rms"] = d["max_norm_dF_over_F_rms"]
        if fp64 is not None:
            r["speedup_vs_fp64"] = round(fp64["seconds"] / mx["seconds"], 3)
        out["mixed"] = r
        del mx
        torch.cuda.empty_cache()
    if "half" in variants:
        log(f"half: {W} warm-up + {K} timed steps")
        r, hf = md_leg(api, torch, s, params, K, W, mode="half", global_format=args.global_format)
        out["half_scatter"] = r
        del hf
        torch.cuda.empty_cache()
    if "c1" in variants:
        log("c1: 4,000 atoms, 100 steps")
        out["c1_4000"] = c1_leg(api, torch, inputs)
    if "c2" in variants:
        log("c2: 256,000 atoms, 1,000 steps, gather and scatter")
        out["c2_256k"] = c2_leg(api, torch, inputs)
    if "large" in variants:
        log("large: 16,384,000 atoms, 1,000 steps, FP64 and mixed")
        out["large_16384k"] = large_leg(api, torch, inputs)
        torch.cuda.empty_cache()
    if "adjoint" in variants:
        log("adjoint: 32,000-atom binary liquid (placement + equilibration first)")
        out["adjoint"] = adjoint_rate(api, torch, inputs)
    if "batch" in variants:
        log("batch: 512 replicas")
        out["batch"] = batch_rates(api, torch, inputs)
    if "sweep" in variants:
        log("sweep: 4,000 to 8,388,608 atoms")
        out["saturation_sweep"] = sweep_rates(api, torch, inputs)
    if not args.no_cpu_baseline:
        log("cpu_baseline: the oracle on one host core")
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
