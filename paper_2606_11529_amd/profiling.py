"""Summaries of rocprofv3 CSV output, and the HBM-traffic record the bench
reads back.

Two inputs come from rocprofv3 runs of the same bench command:
  * ``--kernel-trace --stats``  ->  ``<prefix>_kernel_stats.csv``
  * ``--pmc FETCH_SIZE`` and, in a separate run, ``--pmc WRITE_SIZE``
    ->  ``<prefix>_counter_collection.csv`` (KiB per dispatch).

The byte counters are scaled by what they read for a plain device copy of
known size that the bench performs once before its timed region (256 MiB
read, 256 MiB written): ``factor = true KiB / counted KiB`` per counter.

The traffic record also stores a digest of the kernel sources; the bench
reports a kernel's traffic only while the sources still hash to it, since a
changed kernel makes old counter values meaningless.

    python -m paper_2606_11529_amd.profiling stats  <kernel_stats.csv> [--cmd CMD]
    python -m paper_2606_11529_amd.profiling traffic <fetch.csv> <write.csv> --cmd CMD
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
from typing import Dict, List, Optional

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
CALIB_BYTES = 256 << 20
KIB = 1024


def sources_digest() -> str:
    """SHA-256 over the HIP sources and headers the kernels are built from."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    """Kernel name without its parameter list (``xpr::k_render_bwd<16, 16, 64, 4, false>``)."""
    name = name.replace("void ", "", 1)
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def kernel_stats(path: str) -> List[dict]:
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append({"kernel": short_name(r["Name"]), "calls": int(r["Calls"]),
                         "avg_us": float(r["AverageNs"]) / 1e3,
                         "total_ms": float(r["TotalDurationNs"]) / 1e6,
                         "pct": float(r["Percentage"])})
    return rows


def stats_markdown(path: str, top: int = 25) -> str:
    out = ["| kernel | calls | avg us | total ms | % of GPU time |",
           "|---|---:|---:|---:|---:|"]
    for r in kernel_stats(path)[:top]:
        out.append(f"| `{r['kernel']}` | {r['calls']} | {r['avg_us']:.1f} | "
                   f"{r['total_ms']:.2f} | {r['pct']:.1f} |")
    return "\n".join(out)


def counter_values(path: str, counter: str) -> Dict[str, List[float]]:
    """Per kernel (short name), the counter value of every dispatch, in KiB."""
    acc: Dict[str, List[float]] = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                acc[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return acc


def calibration(values: Dict[str, List[float]]) -> float:
    """true / counted for the 256 MiB copy: the largest dispatch of the
    runtime's device-copy kernel."""
    copies = [v for k, vs in values.items() if "copyBuffer" in k for v in vs]
    if not copies:
        raise ValueError("no device copy dispatch found to calibrate against")
    return (CALIB_BYTES / KIB) / max(copies)


def traffic_table(fetch_csv: str, write_csv: str) -> dict:
    fv = counter_values(fetch_csv, "FETCH_SIZE")
    wv = counter_values(write_csv, "WRITE_SIZE")
    ff, wf = calibration(fv), calibration(wv)
    kernels = {}
    for k in fv:
        if not k.startswith("xpr::"):
            continue
        f = sum(fv[k]) / len(fv[k])
        w = sum(wv.get(k, [0.0])) / max(len(wv.get(k, [])), 1)
        kernels[k] = {"launches": len(fv[k]), "fetch_kib": f, "write_kib": w,
                      "bytes": (f * ff + w * wf) * KIB}
    return {"fetch_factor": ff, "write_factor": wf, "kernels": kernels}


def traffic_text(tab: dict, cmd: str, digest: str) -> str:
    lines = [
        "# HBM traffic per launch from rocprofv3 byte counters",
        f"command: {cmd}",
        "counters: FETCH_SIZE and WRITE_SIZE (KiB per dispatch), one run each",
        f"fetch_factor: {tab['fetch_factor']:.4f}",
        f"write_factor: {tab['write_factor']:.4f}",
        "(factor = true KiB / counted KiB for the bench's 256 MiB device copy)",
        f"sources_sha256: {digest}",
        "",
        f"{'kernel':56s} {'launches':>8s} {'fetch_KiB':>12s} {'write_KiB':>12s} {'bytes':>14s}",
    ]
    rows = sorted(tab["kernels"].items(), key=lambda kv: -kv[1]["bytes"])
    for k, v in rows:
        lines.append(f"{k.replace(' ', ''):56s} {v['launches']:8d} {v['fetch_kib']:12.1f} "
                     f"{v['write_kib']:12.1f} {v['bytes']:14.0f}")
    return "\n".join(lines) + "\n"


def read_traffic(path: str) -> Optional[dict]:
    """Parse a traffic record; None if missing or made from other sources."""
    if not os.path.exists(path):
        return None
    digest, kernels, table = None, {}, False
    with open(path) as f:
        for line in f:
            line = line.rstrip("\n")
            if line.startswith("sources_sha256:"):
                digest = line.split(":", 1)[1].strip()
            elif line.startswith("kernel "):
                table = True
            elif table and line.strip():
                parts = line.split()
                kernels[parts[0]] = float(parts[-1])
    if digest != sources_digest():
        return None
    return kernels


def traffic_of(path: str, kernel: str) -> Optional[float]:
    """Bytes per launch of the kernel whose name starts with ``kernel``
    (template arguments without spaces), or None."""
    tab = read_traffic(path)
    if not tab:
        return None
    key = kernel.replace(" ", "")
    for k, v in tab.items():
        if k == key or k.startswith(key):
            return v
    return None


def valu_busy_of(path: str, kernel: str) -> Optional[float]:
    """The counter-based VALU busy fraction of ``kernel`` (template arguments
    without spaces) from a committed instruction-mix summary (a markdown
    table with a "VALU busy" column), or None when the file is missing, has
    no such row, or was taken from other kernel sources than the current
    ones (its ``sources_sha256:`` line)."""
    try:
        with open(path) as f:
            lines = f.read().splitlines()
    except OSError:
        return None
    digest = next((ln.split(":", 1)[1].strip() for ln in lines
                   if ln.startswith("sources_sha256:")), None)
    if digest != sources_digest():
        return None
    header = None
    key = kernel.replace(" ", "")
    for ln in lines:
        if not ln.startswith("|"):
            continue
        cells = [c.strip() for c in ln.strip("|").split("|")]
        if "VALU busy" in cells:
            header = cells
            continue
        if header and cells and cells[0].strip("`").replace(" ", "") == key:
            try:
                return float(cells[header.index("VALU busy")])
            except (ValueError, IndexError):
                return None
    return None


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", default="")
    s.add_argument("--top", type=int, default=25)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--cmd", required=True)
    a = ap.parse_args()
    if a.what == "stats":
        if a.cmd:
            print(f"command: {a.cmd}\n")
        print(stats_markdown(a.csv, a.top))
    else:
        print(traffic_text(traffic_table(a.fetch_csv, a.write_csv), a.cmd, sources_digest()),
              end="")


if __name__ == "__main__":
    main()
