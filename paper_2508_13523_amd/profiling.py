"""Turn rocprofv3 result databases into the short summaries kept in profiles/.

    python -m paper_2508_13523_amd.profiling trace DB --out FILE.md --command "..."
        kernel-trace statistics (top kernels by total time) as a markdown table;

    python -m paper_2508_13523_amd.profiling counters FETCH_DB WRITE_DB --atoms N
            [--lanes L] --out FILE.json --command "..."
        HBM traffic of the FP64 gather kernel from one FETCH_SIZE pass and one
        WRITE_SIZE pass, each scaled by what the same counter reads for the 1 GiB
        device copy that `bench.py --calibrate-copy` runs (the copy reads and
        writes exactly 2^30 bytes), averaged over the kernel's dispatches.

Both read the SQLite views rocprofv3 writes (`top_kernels`, `counters_collection`).
"""
import argparse
import hashlib
import json
import os
import sqlite3

ROOT = os.path.dirname(os.path.abspath(__file__))
GATHER_SOURCES = [os.path.join(ROOT, "csrc", f) for f in ("force.hip", "tile.hpp", "common.hpp")]


def gather_kernel(lanes: int) -> str:
    """Demangled name of the FP64 tiled gather with `lanes` lanes per atom."""
    return f"k_force_tile_gather<1, false, false, {lanes}, false>"

COPY_BYTES = float(1 << 30)


def gather_source_hash() -> str:
    """Hash of the sources the FP64 tiled gather kernel is compiled from."""
    h = hashlib.sha256()
    for path in GATHER_SOURCES:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    s = name.replace("ljmd::(anonymous namespace)::", "")
    for cut in ("(ljmd", "(double", "(long", "(int"):
        s = s.split(cut)[0]
    return s if len(s) <= 90 else s[:90] + "..."


def trace_summary(db: str, command: str, top: int = 20) -> str:
    con = sqlite3.connect(db)
    rows = list(con.execute(
        "select name, total_calls, total_duration, average, percentage from top_kernels"))
    lines = ["command: `" + command + "`", "",
             "| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for name, calls, tot, avg, pct in rows[:top]:
        # top_kernels durations are in microseconds
        lines.append(f"| `{_short(name)}` | {calls} | {tot / 1e3:.3f} | {avg:.2f} | {pct:.2f} |")
    return "\n".join(lines) + "\n"


def trace_by_grid(db: str, top: int = 12) -> str:
    """Launches grouped by kernel and grid size (so that launches of one kernel
    on different workloads are told apart), with each kernel's registers and
    LDS as the trace records them."""
    con = sqlite3.connect(db)
    rows = list(con.execute(
        "select name, grid_x, workgroup_x, count(*), sum(duration), avg(duration), "
        "max(vgpr_count), max(accum_vgpr_count), max(sgpr_count), max(lds_size) "
        "from kernels group by name, grid_x, workgroup_x order by sum(duration) desc"))
    lines = ["| kernel | grid (lanes) | workgroup | calls | total ms | avg us | VGPR | AGPR | "
             "SGPR | LDS bytes |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for name, gx, wx, calls, tot, avg, vg, ag, sg, lds in rows[:top]:
        # kernel-trace durations are in nanoseconds
        lines.append(f"| `{_short(name)}` | {gx} | {wx} | {calls} | {tot / 1e6:.3f} | "
                     f"{avg / 1e3:.2f} | {vg} | {ag} | {sg} | {lds} |")
    return "\n".join(lines) + "\n"


def _per_dispatch(db: str, counter: str):
    """{kernel name: [(value, duration ns), ...]} for one counter."""
    con = sqlite3.connect(db)
    out = {}
    for kname, disp, cname, val, dur in con.execute(
            "select kernel_name, dispatch_id, counter_name, value, duration "
            "from counters_collection"):
        if cname != counter:
            continue
        out.setdefault(kname, {})[disp] = (float(val), float(dur))
    return {k: list(v.values()) for k, v in out.items()}


def _copy_reading(per: dict) -> float:
    """Counter value (KiB) of the calibration copy: the largest reading among
    the copy kernels."""
    best = 0.0
    for name, vals in per.items():
        if "copy" in name.lower():
            best = max(best, max(v for v, _ in vals))
    if best <= 0.0:
        raise RuntimeError("no copy dispatch found; run the bench with --calibrate-copy")
    return best


def _kernel_mean(per: dict, kernel: str) -> float:
    vals = [v for name, vs in per.items() if kernel in name for v, _ in vs]
    if not vals:
        raise RuntimeError(f"no dispatch of {kernel}")
    return sum(vals) / len(vals)


def counters_summary(fetch_db: str, write_db: str, atoms: int, lanes: int, command: str) -> dict:
    fetch = _per_dispatch(fetch_db, "FETCH_SIZE")
    write = _per_dispatch(write_db, "WRITE_SIZE")
    f_scale = COPY_BYTES / _copy_reading(fetch)
    w_scale = COPY_BYTES / _copy_reading(write)
    kernel = gather_kernel(lanes)
    fk = _kernel_mean(fetch, kernel)
    wk = _kernel_mean(write, kernel)
    return {
        "kernel": kernel,
        "atoms": atoms,
        "kernel_source_sha256_16": gather_source_hash(),
        "fetch_kib_per_dispatch": fk,
        "write_kib_per_dispatch": wk,
        "copy_bytes_per_fetch_kib": f_scale,
        "copy_bytes_per_write_kib": w_scale,
        "hbm_read_bytes_per_launch": fk * f_scale,
        "hbm_write_bytes_per_launch": wk * w_scale,
        "hbm_bytes_per_launch": fk * f_scale + wk * w_scale,
        "command": command,
    }


def _kernel_counter_means(db: str, kernel: str) -> dict:
    """{counter: mean per dispatch} and the mean duration (ns) of the
    dispatches of `kernel` in one --pmc run."""
    con = sqlite3.connect(db)
    per = {}
    durs = {}
    for kname, disp, cname, val, dur in con.execute(
            "select kernel_name, dispatch_id, counter_name, value, duration "
            "from counters_collection"):
        if kernel not in kname:
            continue
        per.setdefault(cname, {})
        per[cname][disp] = per[cname].get(disp, 0.0) + float(val)
        durs[disp] = float(dur)
    if not durs:
        raise RuntimeError(f"no dispatch of {kernel} in {db}")
    out = {c: sum(v.values()) / len(v) for c, v in per.items()}
    out["duration_ns"] = sum(durs.values()) / len(durs)
    return out


def compare_summary(fetch_db: str, write_db: str, sq_db: str, kernels: list, command: str,
                    f32_db: str = None, cus: int = 256, xcds: int = 8,
                    fp64_peak: float = 78.6e12, fp32_peak: float = 157.3e12) -> str:
    """Per-dispatch counter means of several kernels side by side: HBM bytes
    (FETCH_SIZE / WRITE_SIZE scaled by the 1 GiB copy's readings), L2 atomic
    requests, VALU instructions and their FP64 (and, with f32_db, FP32) share,
    VALU busy fraction (instructions / (compute units x cycles), one wave
    instruction per cycle per compute unit at the full FP64 rate) and FP64
    (FP32) FLOP/s against the vector peak."""
    fetch = _per_dispatch(fetch_db, "FETCH_SIZE")
    write = _per_dispatch(write_db, "WRITE_SIZE")
    f_scale = COPY_BYTES / _copy_reading(fetch)
    w_scale = COPY_BYTES / _copy_reading(write)
    rows = []
    for k in kernels:
        f = _kernel_counter_means(fetch_db, k)
        w = _kernel_counter_means(write_db, k)
        q = _kernel_counter_means(sq_db, k)
        t = q["duration_ns"] * 1e-9
        rd = f["FETCH_SIZE"] * f_scale
        wr = w["WRITE_SIZE"] * w_scale
        cycles = q.get("GRBM_GUI_ACTIVE", 0.0) / xcds
        valu = q.get("SQ_INSTS_VALU", 0.0)
        f64 = sum(q.get(c, 0.0) for c in ("SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_MUL_F64",
                                         "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_TRANS_F64"))
        flops = 64.0 * (2.0 * q.get("SQ_INSTS_VALU_FMA_F64", 0.0) +
                        q.get("SQ_INSTS_VALU_MUL_F64", 0.0) + q.get("SQ_INSTS_VALU_ADD_F64", 0.0))
        f32s, f32f = 0.0, 0.0
        if f32_db:
            h = _kernel_counter_means(f32_db, k)
            f32 = sum(h.get(c, 0.0) for c in ("SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_MUL_F32",
                                             "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_TRANS_F32"))
            f32s = f32 / max(h.get("SQ_INSTS_VALU", 0.0), 1.0)
            f32f = 64.0 * (2.0 * h.get("SQ_INSTS_VALU_FMA_F32", 0.0) +
                           h.get("SQ_INSTS_VALU_MUL_F32", 0.0) +
                           h.get("SQ_INSTS_VALU_ADD_F32", 0.0)) / (h["duration_ns"] * 1e-9)
        rows.append((k, t * 1e6, rd / 1e6, wr / 1e6, (rd + wr) / t / 1e9,
                     w.get("TCC_ATOMIC_sum", 0.0), w.get("TCC_EA0_ATOMIC_sum", 0.0),
                     q.get("TA_FLAT_ATOMIC_WAVEFRONTS_sum", 0.0), valu, f64 / max(valu, 1.0),
                     valu / max(cus * cycles, 1.0), flops / t / fp64_peak, f32s,
                     f32f / fp32_peak))
    lines = ["command: `" + command + "`", "",
             "| kernel | us | HBM read MB | HBM write MB | HBM GB/s | L2 atomic requests | "
             "L2-to-memory atomics | atomic wave instructions | VALU instructions | FP64 share | "
             "VALU busy | FP64 FLOP/s of peak | FP32 share | FP32 FLOP/s of peak |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| `{r[0]}` | {r[1]:.1f} | {r[2]:.1f} | {r[3]:.1f} | {r[4]:.0f} | "
                     f"{r[5]:.3g} | {r[6]:.3g} | {r[7]:.3g} | {r[8]:.3g} | {r[9]:.2f} | "
                     f"{r[10]:.2f} | {r[11]:.3f} | {r[12]:.2f} | {r[13]:.3f} |")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--out", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--by-grid", action="store_true",
                   help="also break the launches down by grid size")
    k = sub.add_parser("compare")
    k.add_argument("fetch_db")
    k.add_argument("write_db")
    k.add_argument("sq_db")
    k.add_argument("--f32-db", default=None)
    k.add_argument("--kernel", action="append", required=True)
    k.add_argument("--out", required=True)
    k.add_argument("--command", required=True)
    c = sub.add_parser("counters")
    c.add_argument("fetch_db")
    c.add_argument("write_db")
    c.add_argument("--atoms", type=int, required=True)
    c.add_argument("--lanes", type=int, default=4)
    c.add_argument("--out", required=True)
    c.add_argument("--command", required=True)
    a = ap.parse_args()
    if a.what == "trace":
        text = trace_summary(a.db, a.command)
        if a.by_grid:
            text += "\nBy kernel and grid size:\n\n" + trace_by_grid(a.db)
        with open(a.out, "w") as fh:
            fh.write(text)
    elif a.what == "compare":
        text = compare_summary(a.fetch_db, a.write_db, a.sq_db, a.kernel, a.command,
                               f32_db=a.f32_db)
        with open(a.out, "w") as fh:
            fh.write(text)
    else:
        res = counters_summary(a.fetch_db, a.write_db, a.atoms, a.lanes, a.command)
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
            fh.write("\n")


if __name__ == "__main__":
    main()
