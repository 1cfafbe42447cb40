"""HBM traffic per launch from two rocprofv3 counter passes.

Reads the counter CSVs of one FETCH_SIZE pass and one WRITE_SIZE pass over
the same command (`bench.py --calibrate-copy ...`), scales each counter by
what it reads for the plain 256 MiB device copy of the calibration (known
bytes), and writes a short text summary with the per-launch traffic of the
step kernels and a hash of the kernel sources, so that a later bench run can
tell whether the kernels still match the counters.

    python -m paper_1603_06188_amd.profile_traffic FETCH.csv WRITE.csv OUT.txt "COMMAND" [KERNELS]

KERNELS (optional): comma-separated kernel-name prefixes to summarize instead
of the explicit step's kernels; their keys keep the template arguments
(k_mid_tile<3, 2, 2> -> k_mid_tile_3_2_2).
"""
from __future__ import annotations

import collections
import csv
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
COPY_KIB = 256 * 1024          # the calibration copy: 256 MiB read and 256 MiB written
STEP_KERNELS = ("k_p2g<", "k_grid_update<", "k_bin_keys_moved<", "k_bin_records<", "k_g2p<")


def source_hash() -> str:
    """sha256 over the library's kernel sources and the public header."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(ROOT, "include", "apic.h"), "rb") as f:
        h.update(b"apic.h\0" + f.read())
    return h.hexdigest()


def _per_kernel(path: str, counter: str):
    per = collections.defaultdict(list)
    copies = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        name = re.sub(r"\(.*", "", r["Kernel_Name"].replace("(anonymous namespace)::", "")).replace("void ", "")
        val = float(r["Counter_Value"])
        if "copyBuffer" in name:
            copies.append((int(r["Grid_Size"]), val))
        else:
            per[name].append(val)
    if not copies:
        raise SystemExit(f"{path}: no copy kernel found for the calibration")
    big = max(g for g, _ in copies)
    calib = [v for g, v in copies if g == big]
    return {k: sum(v) / len(v) for k, v in per.items()}, sum(calib) / len(calib)


def read_summary(path: str):
    """{key: value} of a summary written by this module (values as strings)."""
    out = {}
    with open(path) as f:
        for line in f:
            m = re.match(r"^([A-Za-z0-9_<>, ]+?):\s+(.*)$", line.strip())
            if m:
                out[m.group(1)] = m.group(2)
    return out


def _key(name: str, templated: bool) -> str:
    name = re.sub(r"^.*::", "", name.split("<")[0]) + ("<" + name.split("<", 1)[1] if "<" in name else "")
    if not templated:
        return name.split("<")[0]
    return re.sub(r"[<>, ]+", "_", name).strip("_")


def main(argv):
    fetch_csv, write_csv, out_path, command = argv[1:5]
    select = tuple(argv[5].split(",")) if len(argv) > 5 else None
    fetch, fetch_copy = _per_kernel(fetch_csv, "FETCH_SIZE")
    write, write_copy = _per_kernel(write_csv, "WRITE_SIZE")
    fs, ws = COPY_KIB / fetch_copy, COPY_KIB / write_copy
    lines = [
        "HBM traffic per launch of the step kernels, from rocprofv3 FETCH_SIZE and WRITE_SIZE",
        "(KiB per dispatch, averaged over dispatches), each scaled by its reading for a plain",
        f"device copy of 256 MiB (FETCH read {fetch_copy:.1f} KiB -> scale {fs:.4f};",
        f"WRITE read {write_copy:.1f} KiB -> scale {ws:.4f}).",
        "",
        f"command: {command}",
        f"source_sha256: {source_hash()}",
        f"fetch_scale: {fs:.6f}",
        f"write_scale: {ws:.6f}",
        "",
    ]
    for k in sorted(set(fetch) | set(write)):
        short = _key(k, False) + ("<" + k.split("<", 1)[1] if "<" in k else "")
        if select is not None:
            if not short.startswith(select):
                continue
            key = _key(k, True)
        else:
            if not any(s in k for s in STEP_KERNELS):
                continue
            key = k.split("<")[0].replace("apic::", "")
        fb = fetch.get(k, 0.0) * 1024 * fs
        wb = write.get(k, 0.0) * 1024 * ws
        lines.append(f"{key}_fetch_bytes: {fb:.0f}")
        lines.append(f"{key}_write_bytes: {wb:.0f}")
        lines.append(f"{key}_traffic_bytes: {fb + wb:.0f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main(sys.argv)
