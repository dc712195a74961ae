"""Summarise rocprofv3 results (rocpd SQLite files) for one kernel.

Inputs: a --kernel-trace --stats run, a --pmc FETCH_SIZE run and a --pmc
WRITE_SIZE run of the same workload, plus the same two counters taken on the
library's copy kernel moving a known number of bytes (the calibration: HBM
bytes per counter unit). Output: a short Markdown summary and an entry in a
JSON file of per-launch HBM traffic keyed by kernel, tagged with a digest of
the kernel sources it was measured on.

    python -m paper_1804_01918_amd.profsummary --name k_step_f64_caosoa \\
        --match "k_step<d2q37::PrecF64, d2q37::Layout<3, 16>, true, false>" \\
        --trace T.db --fetch F.db --write W.db --copy-fetch CF.db --copy-write CW.db \\
        --copy-bytes 1241513984 --sites 4194304 --alg-bytes 2483027968 \\
        --cmd "..." --md profiles/x.md --json profiles/traffic.json
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sqlite3
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


CSRC = os.path.join(ROOT, "paper_1804_01918_amd", "csrc")
# Sources of the plain lattice kernels and of the learned ones.
PLAIN_SOURCES = ("lb_model.hpp", "lb_layout.hpp", "lb_collide.hpp", "lb_kernels.hpp", "lb_lattice.hip")
LEARNED_SOURCES = PLAIN_SOURCES + ("lb_learned.hpp", "mlp_common.hpp", "mlp_infer.hpp", "lb_mlp_state.hpp")


def source_digest(files=PLAIN_SOURCES) -> str:
    """Digest of the named files under csrc/ (the sources a kernel is built from)."""
    h = hashlib.sha256()
    for name in sorted(files):
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def _db(path: str) -> sqlite3.Connection:
    if os.path.isdir(path):
        cands = sorted(glob.glob(os.path.join(path, "**", "*.db"), recursive=True))
        if not cands:
            raise FileNotFoundError(f"no .db under {path}")
        path = cands[0]
    return sqlite3.connect(path)


def kernel_durations(trace: str) -> dict[str, list[float]]:
    """Kernel name -> list of durations in microseconds."""
    con = _db(trace)
    out: dict[str, list[float]] = {}
    for name, start, end in con.execute("select name, start, end from kernels"):
        out.setdefault(name, []).append((end - start) / 1e3)
    return out


def counter_per_dispatch(db: str, counter: str) -> dict[str, list[float]]:
    con = _db(db)
    out: dict[str, list[float]] = {}
    for name, value in con.execute(
            "select kernel_name, value from counters_collection where counter_name = ?", (counter,)):
        out.setdefault(name, []).append(float(value))
    return out


def _pick(d: dict, match: str):
    hits = [k for k in d if match in k]
    if not hits:
        raise KeyError(f"no kernel matches {match!r}; have {list(d)[:8]}")
    return hits[0], d[hits[0]]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--name", required=True)
    ap.add_argument("--match", required=True)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-match", default="k_copy16")
    ap.add_argument("--copy-bytes", type=int, default=0)
    ap.add_argument("--sites", type=int, required=True)
    ap.add_argument("--alg-bytes", type=int, required=True)
    ap.add_argument("--cmd", required=True, help="the commands that produced the inputs")
    ap.add_argument("--md", required=True)
    ap.add_argument("--json", required=True)
    ap.add_argument("--sources", choices=("plain", "learned"), default="plain",
                    help="which kernel sources the digest of the entry covers")
    ap.add_argument("--alg-flops", type=float, default=0.0, help="algorithmic matrix-core flops per launch")
    ap.add_argument("--valu", action="append", default=[],
                    help="a --pmc run of SQ_* counters (repeatable, paired with --valu-counters); the "
                         "SQ_INSTS_VALU_{FMA,MUL,ADD,TRANS}_F64/_F32 ones give vector flops")
    ap.add_argument("--valu-counters", action="append", default=[],
                    help="the counter names that run collected (space separated)")
    a = ap.parse_args()
    files = PLAIN_SOURCES if a.sources == "plain" else LEARNED_SOURCES
    digest = source_digest(files)

    durs = kernel_durations(a.trace)
    kname, kd = _pick(durs, a.match)
    avg_us = statistics.fmean(kd)
    lines = [f"# {a.name}: rocprofv3 summary", "", "Commands:", "", "```", a.cmd.strip(), "```", "",
             "## Kernel trace (--kernel-trace --stats)", "",
             "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for name, v in sorted(durs.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| `{name[:110]}` | {len(v)} | {statistics.fmean(v):.2f} | {min(v):.2f} | {max(v):.2f} |")
    lines += ["", f"Dominant kernel `{kname}`: average {avg_us:.2f} us per launch; "
              f"algorithmic bytes per launch {a.alg_bytes} -> {a.alg_bytes / (avg_us * 1e-6) / 1e9:.0f} GB/s.", ""]
    if a.alg_flops:
        lines += [f"Algorithmic matrix-core flops per launch {a.alg_flops:.4g} -> "
                  f"{a.alg_flops / (avg_us * 1e-6) / 1e12:.1f} TFLOP/s.", ""]

    if a.valu and a.valu_counters:
        # Each counter counts wavefront instructions; x64 lanes, FMA = 2 flops
        # (FP32 and FP64 counters; binary16 ones are listed only: a packed
        # instruction does two operations per lane).
        vals = {}
        for run, names in zip(a.valu, a.valu_counters):
            for cname in names.split():
                _, cv = _pick(counter_per_dispatch(run, cname), a.match)
                vals.setdefault(cname, statistics.median(cv))
        flops = 0.0
        for cname, v in vals.items():
            if not (cname.endswith("_F32") or cname.endswith("_F64")):
                continue
            if "_FMA_" in cname:
                flops += 2 * 64 * v
            elif any(k in cname for k in ("_MUL_", "_ADD_", "_TRANS_")):
                flops += 64 * v
        lines += ["## Vector ALU work (--pmc, medians per dispatch)", "", "| counter | per dispatch | per site |",
                  "|---|---|---|"]
        for cname, v in vals.items():
            if cname.startswith("SQ_ACTIVE") or cname in ("SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY"):
                unit = "quad-cycles per 64 sites"   # counted in units of 4 cycles
            elif "CYCLES" in cname:
                unit = "cycles per 64 sites"
            else:
                unit = "lane-ops"
            lines.append(f"| {cname} | {v:.4g} | {64 * v / a.sites:.1f} {unit} |")
        lines += ["", f"Counted vector flops (FMA = 2): {flops / a.sites:.0f} per site, "
                      f"{flops / (avg_us * 1e-6) / 1e12:.2f} TFLOP/s at the traced launch time.", ""]
        valu_flops_per_site = flops / a.sites
    else:
        valu_flops_per_site = None

    entry = {"kernel": kname, "sites": a.sites, "avg_launch_us": avg_us,
             "algorithmic_bytes_per_launch": a.alg_bytes, "source_files": list(files), "source_digest": digest,
             "vector_flops_per_site": valu_flops_per_site}
    if a.fetch and a.write and a.copy_fetch and a.copy_write and a.copy_bytes:
        _, fk = _pick(counter_per_dispatch(a.fetch, "FETCH_SIZE"), a.match)
        _, wk = _pick(counter_per_dispatch(a.write, "WRITE_SIZE"), a.match)
        _, cf = _pick(counter_per_dispatch(a.copy_fetch, "FETCH_SIZE"), a.copy_match)
        _, cw = _pick(counter_per_dispatch(a.copy_write, "WRITE_SIZE"), a.copy_match)
        fk_m, wk_m = statistics.median(fk), statistics.median(wk)
        cf_m, cw_m = statistics.median(cf), statistics.median(cw)
        sf = a.copy_bytes / (cf_m * 1024.0)
        sw = a.copy_bytes / (cw_m * 1024.0)
        read_b, write_b = fk_m * 1024.0 * sf, wk_m * 1024.0 * sw
        entry.update({"fetch_kib_per_dispatch": fk_m, "write_kib_per_dispatch": wk_m,
                      "copy_fetch_kib": cf_m, "copy_write_kib": cw_m, "copy_bytes": a.copy_bytes,
                      "fetch_scale": sf, "write_scale": sw, "hbm_read_bytes": read_b,
                      "hbm_write_bytes": write_b, "hbm_bytes_per_launch": read_b + write_b})
        lines += ["## HBM traffic (--pmc FETCH_SIZE, --pmc WRITE_SIZE; medians per dispatch)", "",
                  "| quantity | value |", "|---|---|",
                  f"| FETCH_SIZE, kernel | {fk_m:.0f} KiB |", f"| WRITE_SIZE, kernel | {wk_m:.0f} KiB |",
                  f"| FETCH_SIZE, copy of {a.copy_bytes} B | {cf_m:.0f} KiB (scale {sf:.4f}) |",
                  f"| WRITE_SIZE, copy of {a.copy_bytes} B | {cw_m:.0f} KiB (scale {sw:.4f}) |",
                  f"| HBM read per launch (scaled) | {read_b:.4g} B |",
                  f"| HBM write per launch (scaled) | {write_b:.4g} B |",
                  f"| HBM total / algorithmic | {(read_b + write_b) / a.alg_bytes:.4f} |", ""]
    lines += [f"Kernel sources ({', '.join(files)}) digest: `{digest}`", ""]
    with open(a.md, "w") as fh:
        fh.write("\n".join(lines))

    rec = {"kernels": {}}
    if os.path.exists(a.json):
        with open(a.json) as fh:
            rec = json.load(fh)
        rec.pop("source_digest", None)
        rec.setdefault("kernels", {})
    rec["kernels"][a.name] = entry
    with open(a.json, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
    print(json.dumps(entry))


if __name__ == "__main__":
    main()
