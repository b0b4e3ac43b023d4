"""Summaries of rocprofv3 output databases (rocpd SQLite) for ``profiles/``.

    python -m paper_2001_05291_amd.profiling trace DB OUT.md --title T --command CMD
    python -m paper_2001_05291_amd.profiling traffic --fetch DB --write DB --kernel RE
        --copy RE --copy-bytes N --algorithmic-bytes N OUT.md --command CMD...
    python -m paper_2001_05291_amd.profiling valu --db DB --kernel RE --workload W OUT.md
        --command CMD

``trace`` writes per-kernel launch statistics (calls, mean / min / max
duration).  ``traffic`` turns the FETCH_SIZE and WRITE_SIZE counters (KiB per
dispatch, summed over the counter instances of a dispatch) of one kernel into
bytes per launch, each scaled by what the same counter reads for a plain copy
kernel of known size, and records the hash of the kernel code it was taken
with (the source with its comments removed and its whitespace collapsed) so
that a stale figure is not reported for changed code.
"""

from __future__ import annotations

import argparse
import hashlib
import os
import re
import sqlite3
import statistics

PKG = os.path.dirname(os.path.abspath(__file__))
SWEEP_SOURCE = os.path.join(PKG, "csrc", "engine.hip")


def strip_comments(src: str) -> str:
    """C++ source without its // and /* */ comments (string and character
    literals kept as they are), every run of whitespace made one space."""
    out = []
    i, n = 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def code_hash(path: str = SWEEP_SOURCE) -> str:
    """Hash of the kernel code: a change to a comment keeps it."""
    with open(path, encoding="utf-8") as f:
        return hashlib.sha256(strip_comments(f.read()).encode()).hexdigest()[:16]


def short_name(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "").replace("fs::", "")
    n = re.sub(r"\(.*\)$", "", n)
    return n.replace("void ", "")


def kernel_stats(db: str):
    con = sqlite3.connect(db)
    rows = con.execute(
        "select name, count(*), avg(duration), min(duration), max(duration), sum(duration) "
        "from kernels group by name order by sum(duration) desc").fetchall()
    con.close()
    return [(short_name(n), c, a / 1e3, lo / 1e3, hi / 1e3, s / 1e6) for n, c, a, lo, hi, s in rows]


def counter_per_dispatch(db: str, kernel_re: str, counter: str, most_used: bool = False):
    """Mean over dispatches of the kernel matching kernel_re of the counter's
    value summed over its instances; also the number of dispatches.  Several
    matching kernels are an error unless most_used, which takes the one
    dispatched most often (the variant the autotuner kept, not its trials)."""
    con = sqlite3.connect(db)
    rows = con.execute(
        "select name, dispatch_id, sum(counter_value) from pmc_events where counter_name = ? "
        "group by dispatch_id, name", (counter,)).fetchall()
    con.close()
    hits = [(short_name(n or ""), v) for n, _, v in rows
            if re.search(kernel_re, short_name(n or ""))]
    if not hits:
        raise SystemExit(f"no {counter} samples for kernels matching {kernel_re!r} in {db}")
    names = sorted({n for n, _ in hits})
    if len(names) > 1:
        if not most_used:
            raise SystemExit(f"{kernel_re!r} matches several kernels in {db}: {names}")
        top = max(names, key=lambda x: sum(1 for n, _ in hits if n == x))
        hits = [(n, v) for n, v in hits if n == top]
    vals = [v for _, v in hits]
    return statistics.fmean(vals), len(vals)


def kernel_name(db: str, kernel_re: str, counter: str) -> str:
    """Name of the most-dispatched kernel matching kernel_re in a counter run."""
    con = sqlite3.connect(db)
    rows = con.execute("select name from pmc_events where counter_name = ? group by dispatch_id, "
                       "name", (counter,)).fetchall()
    con.close()
    names = [short_name(n or "") for (n,) in rows if re.search(kernel_re, short_name(n or ""))]
    return max(set(names), key=names.count)


def write_trace(db: str, out: str, title: str, command: str, copy_re: str | None = None,
                copy_bytes: int = 0):
    lines = [f"# {title}", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | mean (us) | min (us) | max (us) | total (ms) |",
             "|---|---:|---:|---:|---:|---:|"]
    stats = kernel_stats(db)
    for n, c, a, lo, hi, s in stats:
        lines.append(f"| `{n}` | {c} | {a:.2f} | {lo:.2f} | {hi:.2f} | {s:.3f} |")
    if copy_re:
        hits = [x for x in stats if re.search(copy_re, x[0])]
        if len(hits) != 1:
            raise SystemExit(f"{copy_re!r} must match exactly one kernel, got {[h[0] for h in hits]}")
        n, c, a, lo, hi, _ = hits[0]
        lines += ["", f"Plain device copy (`{copy_re}`, {copy_bytes} B read + written): "
                      f"{lo:.1f} us at best -> {copy_bytes / (lo * 1e-6) / 1e9:.0f} GB/s "
                      "(the HBM rate a streaming kernel reaches on this device)"]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def write_traffic(fetch_db: str, write_db: str, kernel_re: str, copy_re: str, copy_bytes: int,
                  algorithmic: int, out: str, commands, workload: str):
    f_k, n_f = counter_per_dispatch(fetch_db, kernel_re, "FETCH_SIZE", most_used=True)
    w_k, n_w = counter_per_dispatch(write_db, kernel_re, "WRITE_SIZE", most_used=True)
    used = kernel_name(fetch_db, kernel_re, "FETCH_SIZE")
    f_c, _ = counter_per_dispatch(fetch_db, copy_re, "FETCH_SIZE")
    w_c, _ = counter_per_dispatch(write_db, copy_re, "WRITE_SIZE")
    f_scale = copy_bytes / (f_c * 1024.0)
    w_scale = copy_bytes / (w_c * 1024.0)
    fetch_b = f_k * 1024.0 * f_scale
    write_b = w_k * 1024.0 * w_scale
    total = fetch_b + write_b
    lines = [f"# HBM traffic of `{kernel_re}` ({workload})", "",
             "Commands:", "", "```", *commands, "```", "",
             f"- kernel measured: `{used}` (the most-dispatched match)",
             f"- FETCH_SIZE per dispatch: {f_k:.1f} KiB over {n_f} dispatches; copy kernel "
             f"(`{copy_re}`, {copy_bytes} B read): {f_c:.1f} KiB -> scale {f_scale:.4f}",
             f"- WRITE_SIZE per dispatch: {w_k:.1f} KiB over {n_w} dispatches; copy kernel "
             f"({copy_bytes} B written): {w_c:.1f} KiB -> scale {w_scale:.4f}",
             f"- scaled fetch {fetch_b:.0f} B + write {write_b:.0f} B per launch",
             f"- algorithmic bytes per launch: {algorithmic} "
             f"(traffic / algorithmic = {total / algorithmic:.3f})", "",
             f"workload: {workload}",
             f"traffic_bytes_per_launch: {total:.0f}",
             f"code_sha256: {code_hash()}"]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    return total


def write_valu(db: str, kernel_re: str, out: str, commands, workload: str):
    """VALU work of one kernel from an SQ_INSTS_VALU counter run: wave-level
    VALU instructions per dispatch (summed over the counter's instances),
    times 64 lanes, as lane-operations per launch."""
    v, n = counter_per_dispatch(db, kernel_re, "SQ_INSTS_VALU", most_used=True)
    used = kernel_name(db, kernel_re, "SQ_INSTS_VALU")
    extra = []
    for ctr in ("SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_WAVES"):
        try:
            x, _ = counter_per_dispatch(db, kernel_re, ctr, most_used=True)
            extra.append(f"- {ctr} per dispatch: {x:.0f}")
        except SystemExit:
            pass
    lines = [f"# VALU work of `{kernel_re}` ({workload})", "",
             "Command:", "", "```", *commands, "```", "",
             f"- kernel measured: `{used}` (the most-dispatched match)",
             f"- SQ_INSTS_VALU per dispatch: {v:.0f} wave instructions over {n} dispatches",
             *extra,
             f"- lane-operations per launch (x 64 lanes): {64 * v:.0f}", "",
             f"workload: {workload}",
             f"valu_lane_ops_per_launch: {64 * v:.0f}",
             f"code_sha256: {code_hash()}"]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    return 64 * v


def read_valu(path: str, workload: str):
    """VALU lane-operations per launch recorded in a summary, or None when it
    is missing, for another workload, or taken with a different kernel
    source."""
    try:
        text = open(path).read()
    except OSError:
        return None
    kv = dict(re.findall(r"^(\w+): (.+)$", text, re.M))
    if kv.get("workload") != workload or kv.get("code_sha256") != code_hash():
        return None
    return float(kv["valu_lane_ops_per_launch"])


def sparse_entry_bytes(C) -> int:
    """Bytes per sorted-list entry: a packed 32-bit (cost << 6 | id) key when
    every cost is below 2^26 - 1, else an int32 cost and a uint8 id."""
    import numpy as np
    return 4 if int(np.asarray(C).max()) < (1 << 26) - 1 else 5


def sparse_sweep_bytes(C, open_ids, width: int = 64, entry_bytes: int | None = None) -> int:
    """Bytes the sparse sweep needs in one iteration at placement open_ids:
    for every block of `width` base ids and every mission, the block's sorted
    list up to and including the first entry not below the mission's
    second-nearest open cost (entry_bytes per entry: 4 packed, 5 unpacked;
    by default what the table allows), plus the mission's state (b1, b2, o1:
    12 B) once per block.  C: host (B, M) int32."""
    import numpy as np
    C = np.asarray(C)
    B, M = C.shape
    rows = C[np.asarray(open_ids)]
    if rows.shape[0] >= 2:
        b2 = np.partition(rows, 1, axis=0)[1].astype(np.int64)
    else:
        b2 = np.full(M, 2**31 - 1, dtype=np.int64)
    nb = (B + width - 1) // width
    entries = 0
    for q in range(nb):
        blk = C[q * width:min(B, (q + 1) * width)]
        below = (blk.astype(np.int64) < b2[None, :]).sum(axis=0)
        entries += int(np.minimum(below + 1, width).sum())
    if entry_bytes is None:
        entry_bytes = sparse_entry_bytes(C)
    return entries * entry_bytes + nb * M * 12


def read_traffic(path: str, workload: str):
    """Traffic per launch recorded in a summary, or None when it is missing,
    for another workload, or taken with a different kernel source."""
    try:
        text = open(path).read()
    except OSError:
        return None
    kv = dict(re.findall(r"^(\w+): (.+)$", text, re.M))
    if kv.get("workload") != workload or kv.get("code_sha256") != code_hash():
        return None
    return float(kv["traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("out")
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--copy", default=None, help="kernel-name regex of the copy probe")
    t.add_argument("--copy-bytes", type=int, default=0, help="bytes it reads plus writes")
    r = sub.add_parser("traffic")
    r.add_argument("out")
    r.add_argument("--fetch", required=True)
    r.add_argument("--write", required=True)
    r.add_argument("--kernel", required=True)
    r.add_argument("--copy", required=True)
    r.add_argument("--copy-bytes", type=int, required=True)
    r.add_argument("--algorithmic-bytes", type=int, required=True)
    r.add_argument("--workload", required=True)
    r.add_argument("--command", action="append", default=[])
    v = sub.add_parser("valu")
    v.add_argument("out")
    v.add_argument("--db", required=True)
    v.add_argument("--kernel", required=True)
    v.add_argument("--workload", required=True)
    v.add_argument("--command", action="append", default=[])
    a = ap.parse_args()
    if a.cmd == "trace":
        write_trace(a.db, a.out, a.title, a.command, a.copy, a.copy_bytes)
    elif a.cmd == "valu":
        write_valu(a.db, a.kernel, a.out, a.command, a.workload)
    else:
        write_traffic(a.fetch, a.write, a.kernel, a.copy, a.copy_bytes, a.algorithmic_bytes,
                      a.out, a.command, a.workload)


if __name__ == "__main__":
    main()
