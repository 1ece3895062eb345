#!/usr/bin/env python
"""Lennard-Jones MD benchmark on one MI355X: neighbor build + 12-6 force +
velocity Verlet at 2,048,000 atoms, FP64 and mixed precision, plus the
half-list scatter variant and the adjoint (force-matching gradient) rate.

Prints one JSON line.  `value` is FP64 throughput in millions of atom-steps
per second over K timed steps (each step: half kick + drift, a neighbor
rebuild every 20 steps, the force evaluation, half kick; thermo every 100
steps).  Inputs are synthetic and resident on the GPU before timing starts.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Matom-steps/s LJ force+neigh @2M atoms: FP64 vs mixed; adjoint grads/s"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
COUNTERS = os.path.join(ROOT, "profiles", "force_gather_fp64_2048k_counters.json")


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--ncell", type=int, default=80, help="FCC cells per side (80 -> 2,048,000 atoms)")
    ap.add_argument("--variants", default="fp64,mixed,half,adjoint,batch")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--global-format", action="store_true",
                    help="build lists in the global (atom-index) format instead of tiled")
    ap.add_argument("--gather-lanes", type=int, default=0,
                    help="lanes per atom of the tiled full-list gather (1, 2, 4; 0: library default)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference dispatch for counters)")
    return ap.parse_args()


def run_md(api, torch, s, params, steps, warmup, mixed=False, mode="full", rebuild=20,
           thermo_every=100, sort=True, global_format=False):
    """Warm-up then K timed steps; returns timing, per-phase GPU time and state."""
    dev = torch.device("cuda")
    x = torch.tensor(s.x, device=dev)
    v = torch.tensor(s.v, device=dev)
    f = torch.zeros_like(x)
    cap = api.default_capacity(params, s.box, s.n)
    nl = api.NeighborList(s.n, cap, s.box, params, mode=mode, global_format=global_format)
    ws = api.workspace(s.n, s.box, params)
    api.md_step(x, v, f, None, s.box, params, nl, s.dt, warmup, step0=0, rebuild_every=rebuild,
                setup=True, mixed=mixed, ws=ws, sort=sort)
    st = api.get_status(nl)
    if st[0]:
        raise RuntimeError(f"neighbor capacity {cap} exceeded in warm-up (need {st[1]})")
    rows = api.thermo_rows(warmup, steps, thermo_every, False)
    thermo = torch.zeros((max(rows, 1), 9), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    api.profile_read()
    api.profile_enable(True)
    t0 = time.perf_counter()
    api.md_step(x, v, f, None, s.box, params, nl, s.dt, steps, step0=warmup, rebuild_every=rebuild,
                thermo_every=thermo_every, mixed=mixed, ws=ws, thermo=thermo, sort=sort)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.profile_enable(False)
    phases = api.profile_read()
    st = api.get_status(nl)
    if st[0]:
        raise RuntimeError(f"neighbor capacity {cap} exceeded (need {st[1]})")
    nbar = float(nl.numneigh[: s.n].to(torch.float64).mean().item())
    return dict(seconds=t1 - t0, phases=phases, status=st.tolist(), nbar=nbar, x=x, v=v, f=f,
                nl=nl, thermo=thermo[:rows], ws=ws, format=nl.format, tile=list(nl.tile))


def roofline(N, nbar, phases, fmt, lanes, fused):
    """Force gather kernel: algorithmic bytes per launch = N (4 + e nbar + 24 + 24):
    the row length, the row's neighbor entries (e = 2 bytes per entry in the tiled
    format, 4 in the global one), x_i and f_i; in the MD step with a tiled full
    list the kernel also applies the velocity-Verlet update, which adds 72 bytes
    per atom (read and write v_i, write the drifted x_i)."""
    ms, launches = phases["force"]
    avg_ms = ms / max(launches, 1)
    entry = 2.0 if fmt == "tiled" else 4.0
    per_atom = 4.0 + entry * nbar + 24.0 + 24.0 + (72.0 if fused else 0.0)
    bytes_per_launch = N * per_atom
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
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
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": (f"k_force_tile_gather<1,false,false,{lanes},false>" if fmt == "tiled" else
                       "k_force_gather<1,false,false>") + " (FP64 full-list gather" +
                      (", fused velocity-Verlet update)" if fused else ")"),
            "algorithmic_bytes_per_atom": round(per_atom, 2),
            "avg_launch_ms": round(avg_ms, 5), "launches": launches,
            "algorithmic_bytes_per_launch": int(bytes_per_launch),
            "mean_neighbors": round(nbar, 3)}


def cpu_baseline(s, steps):
    """The oracle (serial C, FP64, Verlet list rebuilt every 20 steps) on the same
    2,048,000-atom system: time of (set-up + `steps` steps) minus time of set-up
    alone = one list build plus `steps` force/integration steps."""
    from oracle import ljref

    ljref.lib()
    t0 = time.perf_counter()
    ljref.md(s.x, s.v, None, s.box, s.eps, s.sigma, s.rc, s.mass, s.dt, 0, rebuild_every=20,
             skin=s.skin)
    t1 = time.perf_counter()
    ljref.md(s.x, s.v, None, s.box, s.eps, s.sigma, s.rc, s.mass, s.dt, steps, rebuild_every=20,
             skin=s.skin)
    t2 = time.perf_counter()
    per = (t2 - t1) - (t1 - t0)
    return {"value": round(s.n * steps / per / 1e6, 4), "unit": "Matom-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{s.n} atoms, {steps} steps incl. one list rebuild (set-up timed "
                      f"separately and subtracted); {t2 - t0:.1f} s of CPU work"}


def adjoint_rate(api, torch, inputs, evals=200):
    """Force-matching gradient evaluations per second on a 32,000-atom binary
    liquid: forward F, loss gradient g = 2 (F - F_t) / N, adjoint to x, eps, sigma.
    Timed eagerly (one library call per kernel) and with the whole evaluation
    captured once in a HIP graph and replayed; every replay's gradients are
    checked against the eager ones; grads_per_s is the faster of the two."""
    s = inputs.binary_liquid(32000, seed=3)
    params = api.LJParams.from_system(s)
    dev = torch.device("cuda")
    x = torch.tensor(s.x, device=dev)
    t = torch.tensor(s.types, device=dev, dtype=torch.int32)
    nl = api.build_list(x, t, s.box, params)
    # the atoms put into cell order once, untimed (the order the MD keeps by
    # sorting at each rebuild); the list is rebuilt with it
    api.md_step(x, torch.tensor(s.v, device=dev), torch.empty_like(x), t, s.box, params, nl,
                s.dt, 0, setup=True, sort=True)
    e_t, s_t = inputs.perturbed_params(s.eps, s.sigma, seed=4)
    ft, _ = api.lj_forces(x, t, s.box, api.LJParams(e_t, s_t, s.rc, s.skin), nl)
    ws = api.workspace(s.n, s.box, params)
    f = torch.empty_like(x)
    g = torch.empty_like(x)

    def grad():
        api.lj_forces(x, t, s.box, params, nl, f=f, ws=ws)
        torch.sub(f, ft, out=g).mul_(2.0 / s.n)
        return api.lj_backward(x, t, s.box, params, nl, g, ws=ws)

    for _ in range(5):
        ref = grad()
    ref = [r.clone() for r in ref]
    torch.cuda.synchronize()
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
            "workload": "binary LJ 80:20, 32,000 atoms, rho 1.2, FP64 forward + adjoint to "
                        "positions and the 2x2 eps/sigma tables; atoms in cell order (sorted "
                        "once before timing); the faster of eager calls and one HIP graph per "
                        "evaluation"}


def batch_rates(api, torch, inputs, replicas=512, iters=20, md_steps=100):
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
    # every system's atoms put into cell order once, untimed (the order the
    # MD below keeps by sorting at each rebuild); the list is rebuilt with it
    B.md_step(x, v, torch.empty_like(x), t, bt, prm, nl, 0.005, 0, setup=True, mixed=True,
              sort=True, ws=ws)
    x0, v0 = x.clone(), v.clone()
    e_t, s_t = inputs.perturbed_params(rb["eps"], rb["sigma"], seed=4)
    prm_t = api.LJParams(e_t, s_t, rb["rc"], rb["skin"], rb["mass"])
    ft, _ = B.lj_forces(x, t, bt, prm_t, nl, ws=ws)
    # loss = sum_r (1/N_r) sum_i |F_i - F_t,i|^2  ->  g_i = 2 (F_i - F_t,i) / N_r
    scale = torch.tensor(np.repeat(2.0 / sizes.astype(np.float64), sizes)[:, None], device=dev)
    tuning = B.autotune(x, t, bt, prm, nl, mixed=True, ws=ws)
    f = torch.empty_like(x)

    def batched():
        B.lj_forces(x, t, bt, prm, nl, mixed=True, f=f, ws=ws)
        g = (f - ft).mul_(scale)
        return B.lj_backward(x, t, bt, prm, nl, g, ws=ws)

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
    # rebuild
    x.copy_(x0)
    v.copy_(v0)
    fm = torch.zeros_like(x)
    nlm = B.neighbor_list(bt, prm, nl.cap)
    B.md_step(x, v, fm, t, bt, prm, nlm, 0.005, 0, setup=True, mixed=True, sort=True, ws=ws)
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            B.md_step(x, v, fm, t, bt, prm, nlm, 0.005, md_steps, step0=0, rebuild_every=20,
                      mixed=True, sort=True, ws=ws)
    torch.cuda.current_stream().wait_stream(st)
    g.replay()
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
                       "persistent": tuning[2]},
            "replica_grads_per_s": round(replicas / t_batch, 1),
            "atom_grads_per_s": round(n / t_batch, 1),
            "ms_per_batch_grad": round(t_batch * 1e3, 4),
            "sequential_fp64_ms_per_batch_grad": round(t_seq * 1e3, 4),
            "speedup_vs_sequential": round(t_seq / t_batch, 2),
            "md_graph_matom_steps_per_s": round(n / t_md / 1e6, 2),
            "md_graph_ms_per_step": round(t_md * 1e3, 4),
            "md_status_overflow": int(stat[0]),
            "workload": "512 binary LJ 80:20 replicas, N_r uniform on [500, 8000], rho 1.2, "
                        "mixed forward + FP64 adjoint per force-matching gradient; MD with "
                        "rebuild every 20 captured in one HIP graph; atoms in cell order "
                        "(sorted once before the gradients, at every rebuild in the MD)"}


def large_rates(api, torch, inputs, steps=1000, warmup=50, ncell=160):
    """16,384,000 atoms (160^3 FCC cells), FP64 and mixed precision, each
    `steps` steps with rebuild every 20: throughput, the mixed force error at
    identical positions, and each run's energy drift."""
    s16 = inputs.fcc_liquid(ncell)
    p16 = api.LJParams.from_system(s16)
    n = s16.n
    res = {"atoms": n, "steps": steps}
    runs = {}
    for name, mixed in (("fp64", False), ("mixed", True)):
        r = run_md(api, torch, s16, p16, steps, warmup, mixed=mixed, thermo_every=100)
        th = r["thermo"].cpu().numpy()
        e = th[:, 1] + th[:, 2]
        runs[name] = r
        res[name] = {"value": round(n * steps / r["seconds"] / 1e6, 2),
                     "ms_per_step": round(r["seconds"] / steps * 1e3, 4),
                     "force_kernel_ms": round(r["phases"]["force"][0] /
                                              max(r["phases"]["force"][1], 1), 5),
                     "energy_drift_per_atom": float(abs(e[-1] - e[0]) / n),
                     "max_energy_excursion_per_atom": float(np.abs(e - e[0]).max() / n)}
        if name == "fp64":
            del r["x"], r["v"], r["f"]
            torch.cuda.empty_cache()
    mx = runs["mixed"]
    f64, _ = api.lj_forces(mx["x"], None, s16.box, p16, mx["nl"], ws=mx["ws"])
    f32, _ = api.lj_forces(mx["x"], None, s16.box, p16, mx["nl"], mixed=True, ws=mx["ws"])
    d = (f32 - f64).abs()
    res["mixed"]["max_abs_dF_over_max_abs_F"] = float(d.max() / f64.abs().max())
    res["mixed"]["max_norm_dF_over_F_rms"] = float(d.norm(dim=1).max() /
                                                   f64.norm(dim=1).pow(2).mean().sqrt())
    res["mixed"]["speedup_vs_fp64"] = round(res["mixed"]["value"] / res["fp64"]["value"], 3)
    return res


def sweep_rates(api, torch, inputs, cells=(10, 16, 20, 26, 32, 40, 50, 64, 80, 100, 128, 160)):
    """Saturation sweep: MD throughput (rebuild every 20, atoms sorted into
    cell order) from 4,000 to 16,384,000 atoms: full list in FP64 and mixed,
    and the FP64 half list (Newton's third law, forces by scatter), so that
    the two list styles can be compared at every size; with the mean time of
    the force phase.  About 40 ms of timed full-list steps per size (100 to
    2,000 steps; the half list runs as many steps)."""
    rows = []
    for nc in cells:
        s = inputs.fcc_liquid(nc)
        p = api.LJParams.from_system(s)
        row = {"fcc_cells": nc, "atoms": s.n}
        for name, mixed, mode in (("fp64", False, "full"), ("mixed", True, "full"),
                                  ("half_fp64", False, "half")):
            steps = min(2000, max(100, int(4e-2 / (s.n * 1.6e-10)) // 20 * 20))
            r = run_md(api, torch, s, p, steps, 20, mixed=mixed, mode=mode, thermo_every=0)
            f = r["phases"].get("force", (0.0, 0))
            row[name] = {"Matom_steps_per_s": round(s.n * steps / r["seconds"] / 1e6, 2),
                         "us_per_step": round(r["seconds"] / steps * 1e6, 2),
                         "force_phase_us": round(f[0] / max(f[1], 1) * 1e3, 2), "steps": steps}
            del r
            torch.cuda.empty_cache()
        if s.n <= 300_000:
            row["fp64_graph"] = graph_md_rate(api, torch, s, p)
        print(f"sweep {nc}^3 cells, {s.n} atoms: {row['fp64']['Matom_steps_per_s']} / "
              f"{row['mixed']['Matom_steps_per_s']} / {row['half_fp64']['Matom_steps_per_s']} "
              "Matom-steps/s (FP64 / mixed / FP64 half list)"
              + (f", {row['fp64_graph']['Matom_steps_per_s']} FP64 graph-replayed"
                 if "fp64_graph" in row else ""),
              file=sys.stderr, flush=True)
        rows.append(row)
    return rows


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


def main():
    args = parse()
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
                                  "sorted into cell order, thermo every 100",
                      "atoms": N, "rebuild_every": 20, "list": "full"}}

    fp64 = None
    if "fp64" in variants:
        fp64 = run_md(api, torch, s, params, K, W, global_format=args.global_format)
        out["value"] = round(N * K / fp64["seconds"] / 1e6, 2)
        out["ms_per_step"] = round(fp64["seconds"] / K * 1e3, 4)
        out["phases_ms_per_step"] = {k: round(v[0] / K, 5) for k, v in fp64["phases"].items()}
        lanes = api.nl_gather_lanes(fp64["nl"], s.box, params)
        out["roofline"] = roofline(N, fp64["nbar"], fp64["phases"], fp64["format"], lanes,
                                   fused=fp64["format"] == "tiled")
        out["config"]["list_format"] = fp64["format"]
        out["config"]["gather_lanes_per_atom"] = lanes
        out["config"]["tile_cells"] = fp64["tile"]
        th = fp64["thermo"].cpu().numpy()
        if th.shape[0] >= 2:
            out["fp64_energy_drift_per_atom"] = float(abs((th[-1, 1] + th[-1, 2]) -
                                                          (th[0, 1] + th[0, 2])) / N)
        out["dangerous_builds_flagged"] = bool(fp64["status"][2])
    if "mixed" in variants:
        mx = run_md(api, torch, s, params, K, W, mixed=True, global_format=args.global_format)
        r = {"value": round(N * K / mx["seconds"] / 1e6, 2),
             "ms_per_step": round(mx["seconds"] / K * 1e3, 4),
             "force_kernel_ms": round(mx["phases"]["force"][0] / max(mx["phases"]["force"][1], 1), 5)}
        # force error at identical positions: mixed vs FP64 on the mixed run's final state
        f64, _ = api.lj_forces(mx["x"], None, s.box, params, mx["nl"], ws=mx["ws"])
        f32, _ = api.lj_forces(mx["x"], None, s.box, params, mx["nl"], mixed=True, ws=mx["ws"])
        d = (f32 - f64).abs()
        r["max_abs_dF_over_max_abs_F"] = float(d.max() / f64.abs().max())
        r["max_norm_dF_over_F_rms"] = float(d.norm(dim=1).max() / f64.norm(dim=1).pow(2).mean().sqrt())
        th = mx["thermo"].cpu().numpy()
        if th.shape[0] >= 2:
            r["energy_drift_per_atom"] = float(abs((th[-1, 1] + th[-1, 2]) -
                                                   (th[0, 1] + th[0, 2])) / N)
        if fp64 is not None:
            r["speedup_vs_fp64"] = round(fp64["seconds"] / mx["seconds"], 3)
        out["mixed"] = r
        del mx
    if "half" in variants:
        hf = run_md(api, torch, s, params, K, W, mode="half", global_format=args.global_format)
        out["half_scatter"] = {
            "value": round(N * K / hf["seconds"] / 1e6, 2),
            "ms_per_step": round(hf["seconds"] / K * 1e3, 4),
            "force_kernel_ms": round(hf["phases"]["force"][0] / max(hf["phases"]["force"][1], 1), 5),
            "mean_neighbors": round(hf["nbar"], 3)}
        del hf
    if "adjoint" in variants:
        out["adjoint"] = adjoint_rate(api, torch, inputs)
    if "batch" in variants:
        out["batch"] = batch_rates(api, torch, inputs)
    if "large" in variants:
        out["large_16384k"] = large_rates(api, torch, inputs)
    if "sweep" in variants:
        out["saturation_sweep"] = sweep_rates(api, torch, inputs)
    if fp64 is not None:
        del fp64
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
