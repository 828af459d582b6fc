"""Short text summaries of rocprofv3 output (its SQLite ``*_results.db``).

    # per-kernel durations of a --kernel-trace run (optionally only kernels whose
    # name contains MATCH, and one row per launch grid)
    python -m paper_1601_05448_amd.profile_summary stats DIR [--top 20] [--match MATCH] [--by-grid]

    # HBM bytes per launch of one kernel from a FETCH_SIZE run and a WRITE_SIZE
    # run, each scaled by what the counter reads for a device copy of known size
    python -m paper_1601_05448_amd.profile_summary traffic --fetch DIR --write DIR \\
        --kernel 'k_resid_dhtx_z<float, 256' --key f32:k_resid_dhtx_z@256 --copy-mib 1024 \\
        --json profiles/traffic.json

    # HBM bytes per cell of every kernel from the same two runs
    python -m paper_1601_05448_amd.profile_summary bytes --fetch DIR --write DIR --cells 16777216

    # per-solve breakdown of a --kernel-trace run (a solve starts at k_init):
    # span, kernel time, gaps, and launches per kernel with the idle ones apart
    python -m paper_1601_05448_amd.profile_summary solves DIR [--first K] [--count N] [--min-kernels M]

The traffic record carries a hash of the kernel sources, so that a reader can
tell counters taken on older code from current ones.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sqlite3
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("poisson_sweeps.hip", "poisson_device.hpp", "poisson_fft.hpp", "poisson_internal.hpp",
                  "poisson_kernels.hip", "poisson_control.hpp")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def _db(d: str) -> sqlite3.Connection:
    files = sorted(glob.glob(os.path.join(d, "**", "*.db"), recursive=True))
    if not files:
        raise SystemExit(f"no rocprofv3 database under {d}")
    return sqlite3.connect(files[0])


def kernel_durations(d: str, by_grid: bool = False) -> dict:
    """kernel name (with the launch grid in work-items when by_grid) -> list of
    dispatch durations (ns)."""
    out: dict = {}
    q = "select name, duration, grid_x, grid_y, grid_z from kernels"
    for name, dur, gx, gy, gz in _db(d).execute(q):
        key = f"[grid {gx}x{gy}x{gz}] {name}" if by_grid else name
        out.setdefault(key, []).append(float(dur))
    return out


def counter_values(d: str, counter: str) -> dict:
    """kernel name -> list of per-dispatch values of `counter` (summed over the
    dispatch's instances)."""
    per: dict = {}
    q = "select dispatch_id, kernel_name, value from counters_collection where counter_name = ?"
    for disp, name, val in _db(d).execute(q, (counter,)):
        key = (disp, name)
        per[key] = per.get(key, 0.0) + float(val)
    out: dict = {}
    for (_, name), v in per.items():
        out.setdefault(name, []).append(v)
    return out


def cmd_stats(a) -> None:
    durs = kernel_durations(a.dir, a.by_grid)
    total = sum(sum(v) for v in durs.values())
    rows = sorted(((k, v) for k, v in durs.items() if a.match in k), key=lambda kv: -sum(kv[1]))[: a.top]
    print(f"{'calls':>6} {'total_ms':>9} {'avg_us':>8} {'min_us':>8} {'max_us':>8} {'pct':>6}  kernel")
    for name, v in rows:
        print(f"{len(v):6d} {sum(v) / 1e6:9.3f} {statistics.fmean(v) / 1e3:8.1f} {min(v) / 1e3:8.1f} "
              f"{max(v) / 1e3:8.1f} {100 * sum(v) / total:6.2f}  {name[:150]}")


def _pick(values: dict, match: str) -> tuple:
    names = [n for n in values if match in n]
    if not names:
        raise SystemExit(f"no kernel matching {match!r}; have: {sorted(values)[:20]}")
    vals = [x for n in names for x in values[n]]
    return names, vals


def cmd_traffic(a) -> None:
    copy_bytes = a.copy_mib * (1 << 20)
    res = {}
    for counter, d in (("FETCH_SIZE", a.fetch), ("WRITE_SIZE", a.write)):
        vals = counter_values(d, counter)
        _, copies = _pick(vals, a.copy_kernel)
        copy_kib = max(copies)  # the 1 GiB copy is the largest dispatch of its kernel
        scale = (copy_bytes / 1024.0) / copy_kib
        names, kv = _pick(vals, a.kernel)
        # launches that did their work (an idle launch reads a few KiB)
        big = [x for x in kv if x > 0.1 * max(kv)]
        kib = statistics.median(big)
        res[counter] = dict(kib_per_launch=kib, launches=len(big), copy_kib=copy_kib, scale=scale,
                            bytes_per_launch=kib * 1024.0 * scale, kernels=names)
    total = res["FETCH_SIZE"]["bytes_per_launch"] + res["WRITE_SIZE"]["bytes_per_launch"]
    for counter, r in res.items():
        print(f"{counter}: {r['kib_per_launch']:.0f} KiB per launch (median of {r['launches']}), copy of "
              f"{a.copy_mib} MiB reads {r['copy_kib']:.0f} KiB -> scale {r['scale']:.4f} -> "
              f"{r['bytes_per_launch'] / 1e6:.1f} MB per launch")
    print(f"HBM traffic per launch: {total / 1e6:.1f} MB ({a.key})")
    if a.json:
        try:
            with open(a.json) as f:
                db = json.load(f)
        except (OSError, ValueError):
            db = {}
        db[a.key] = dict(bytes_per_launch=total, fetch_bytes=res["FETCH_SIZE"]["bytes_per_launch"],
                         write_bytes=res["WRITE_SIZE"]["bytes_per_launch"],
                         fetch_scale=res["FETCH_SIZE"]["scale"], write_scale=res["WRITE_SIZE"]["scale"],
                         kernels=res["FETCH_SIZE"]["kernels"], source_sha256=kernel_source_hash())
        with open(a.json, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
            f.write("\n")


def cmd_bytes(a) -> None:
    """HBM bytes per grid cell read and written by every kernel, each counter
    scaled by the copy kernel's reading (working launches only)."""
    copy_kib = a.copy_mib * 1024.0
    f = counter_values(a.fetch, "FETCH_SIZE")
    w = counter_values(a.write, "WRITE_SIZE")
    fs = copy_kib / max(_pick(f, a.copy_kernel)[1])
    ws = copy_kib / max(_pick(w, a.copy_kernel)[1])
    print(f"scales: FETCH_SIZE x{fs:.4f}, WRITE_SIZE x{ws:.4f} (copy of {a.copy_mib} MiB); cells {a.cells}")
    print(f"{'read B/cell':>11} {'write B/cell':>12}  kernel")
    for name in sorted(f, key=lambda n: -max(f[n])):
        fv = [x for x in f[name] if x > 0.1 * max(f[name])]
        wl = w.get(name, [0.0])
        wv = [x for x in wl if x >= 0.1 * max(wl)] or [0.0]
        if max(fv) * fs * 1024 < 0.5 * a.cells:
            continue
        print(f"{statistics.median(fv) * fs * 1024 / a.cells:11.2f} {statistics.median(wv) * ws * 1024 / a.cells:12.2f}"
              f"  {name[:110]}")


SWEEP_KERNELS = ("k_resid_dhtx_z", "k_dht_cols", "k_dht_z_solve", "k_dhtx_update", "k_outer_resid_dhtx",
                 "k_outer_update")


def cmd_solves(a) -> None:
    """Solves in launch order (each from one k_init to the next): kernels, span
    from the first start to the last end, time inside kernels, gaps between
    them, and per kernel the launches and time, a sweep launch shorter than
    `idle_us` counted apart as idle (its solve was finished or out of stage)."""
    q = "select name, start, end from kernels order by start"
    rows = [(n, s, e) for n, s, e in _db(a.dir).execute(q) if "pois::" in n]
    inits = [i for i, r in enumerate(rows) if "k_init" in r[0]]
    segs = [(si, rows[i:inits[si + 1] if si + 1 < len(inits) else len(rows)]) for si, i in enumerate(inits)]
    # solves of at least min_kernels launches (the sweep timings of the profile
    # driver also start at k_init, with a handful of launches)
    segs = [(si, seg) for si, seg in segs if len(seg) >= getattr(a, "min_kernels", 0)]
    for si, seg in segs[a.first:a.first + a.count]:
        span = (seg[-1][2] - seg[0][1]) / 1e3
        busy = sum(e - s for _, s, e in seg) / 1e3
        per: dict = {}
        for n, s, e in seg:
            base = n.split("(")[0].replace("void ", "").replace("pois::", "").split("<")[0]
            idle = base in SWEEP_KERNELS and (e - s) / 1e3 < a.idle_us
            key = base + (" (idle)" if idle else "")
            c = per.setdefault(key, [0, 0.0])
            c[0] += 1
            c[1] += (e - s) / 1e3
        print(f"solve {si}: {len(seg)} kernels, span {span:.1f} us, in kernels {busy:.1f} us, "
              f"gaps {span - busy:.1f} us")
        for key, (cnt, t) in sorted(per.items(), key=lambda kv: -kv[1][1]):
            print(f"  {cnt:4d} {t:9.1f} us  {key}")


def main(argv=None) -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--top", type=int, default=20)
    s.add_argument("--match", default="", help="only kernels whose name contains this")
    s.add_argument("--by-grid", action="store_true", help="one row per kernel and launch grid")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True, help="substring of the kernel name")
    t.add_argument("--key", required=True)
    t.add_argument("--copy-kernel", default="copy", help="substring of the copy kernel's name")
    t.add_argument("--copy-mib", type=int, default=1024)
    t.add_argument("--json", default="")
    v = sub.add_parser("solves")
    v.add_argument("dir")
    v.add_argument("--first", type=int, default=0, help="index of the first solve shown")
    v.add_argument("--count", type=int, default=4)
    v.add_argument("--idle-us", type=float, default=6.0)
    v.add_argument("--min-kernels", type=int, default=0, help="only solves of at least this many launches")
    b = sub.add_parser("bytes")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--cells", type=int, required=True)
    b.add_argument("--copy-kernel", default="copy")
    b.add_argument("--copy-mib", type=int, default=1024)
    a = ap.parse_args(argv)
    {"stats": cmd_stats, "traffic": cmd_traffic, "bytes": cmd_bytes, "solves": cmd_solves}[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
