"""Summarise rocprofv3 output of the hPF-MD step into profiles/.

python -m paper_1310_2041_amd.profile_summary --stats DIR --fetch DIR --write DIR
       --command "..." --pmc-command "..." --out profiles/NAME.md

--stats  directory of a `--kernel-trace --stats --output-format csv` run
--fetch / --write  directories of `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of
         `python -m paper_1310_2041_amd.profile_step` (which ends with a 1 GiB copy)
The summary ends with a fenced JSON record holding, per kernel, the average
duration and the HBM bytes per launch (counter KiB scaled by the copy
calibration), plus a hash of the kernel sources so that stale traffic is not
reported after a kernel changes; `read_record` parses it back.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30


def source_hash() -> str:
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(HERE, "csrc", "*"))) + [
        os.path.join(os.path.dirname(HERE), "include", "hpf.h")]
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").strip()


def kernel_stats(d: str) -> dict:
    path = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if not path:
        raise SystemExit(f"no kernel_stats.csv under {d}")
    out = {}
    for r in csv.DictReader(open(path[0])):
        out[_short(r["Name"])] = {"calls": int(r["Calls"]), "avg_us": float(r["AverageNs"]) / 1e3,
                                  "total_us": float(r["TotalDurationNs"]) / 1e3,
                                  "pct": float(r["Percentage"])}
    return out


def counter(d: str, name: str):
    """Per-kernel average of counter `name` per dispatch, and (kernel, value) of the
    run's last dispatch, which the profiled program makes the calibration copy."""
    path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not path:
        raise SystemExit(f"no counter_collection.csv under {d}")
    per = collections.defaultdict(float)
    kname = {}
    for r in csv.DictReader(open(path[0])):
        if r["Counter_Name"] != name:
            continue
        i = int(r["Dispatch_Id"])
        per[i] += float(r["Counter_Value"])
        kname[i] = _short(r["Kernel_Name"])
    agg = collections.defaultdict(list)
    for i, v in per.items():
        agg[kname[i]].append(v)
    last = max(per)
    return {k: sum(v) / len(v) for k, v in agg.items()}, (kname[last], per[last])


def read_record(path: str):
    """The JSON record at the end of a summary written by this module, or None."""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    i = txt.rfind("```json\n")
    if i < 0:
        return None
    j = txt.find("```", i + 8)
    return json.loads(txt[i + 8:j])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--pmc-command", required=True)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    stats = kernel_stats(args.stats)
    fetch, (ck, f_copy) = counter(args.fetch, "FETCH_SIZE")
    write, (wk, w_copy) = counter(args.write, "WRITE_SIZE")
    if "copy" not in ck.lower() or wk != ck:
        raise SystemExit(f"last dispatch is {ck} / {wk}, not the calibration copy")
    f_scale = COPY_BYTES / (f_copy * 1024.0)
    w_scale = COPY_BYTES / (w_copy * 1024.0)
    rows = []
    for k, st in sorted(stats.items(), key=lambda kv: -kv[1]["total_us"]):
        rb = fetch.get(k)
        wb = write.get(k)
        rows.append({"kernel": k, **st,
                     "fetch_bytes": rb * 1024.0 * f_scale if rb is not None else None,
                     "write_bytes": wb * 1024.0 * w_scale if wb is not None else None})
    lines = [f"# rocprofv3 summary: {os.path.basename(args.out).rsplit('.', 1)[0]}", "",
             "Kernel trace command:", "", f"    {args.command}", "",
             "Counter commands (one pass each, FETCH_SIZE then WRITE_SIZE):", "",
             f"    {args.pmc_command}", "",
             f"Counter calibration with a plain {COPY_BYTES >> 20} MiB copy ({ck}): "
             f"FETCH_SIZE x{f_scale:.3f}, WRITE_SIZE x{w_scale:.3f} (true bytes per reported byte).",
             f"Kernel source hash: {source_hash()}", "",
             "| kernel | calls | avg us | share % | HBM read MB/launch | HBM write MB/launch |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        fm = f"{r['fetch_bytes'] / 1e6:.1f}" if r["fetch_bytes"] is not None else "-"
        wm = f"{r['write_bytes'] / 1e6:.1f}" if r["write_bytes"] is not None else "-"
        lines.append(f"| {r['kernel']} | {r['calls']} | {r['avg_us']:.2f} | {r['pct']:.1f} | {fm} | {wm} |")
    rec = {"source_hash": source_hash(), "fetch_scale": f_scale, "write_scale": w_scale,
           "kernels": {r["kernel"]: {"avg_us": round(r["avg_us"], 3),
                                     "fetch_bytes": r["fetch_bytes"], "write_bytes": r["write_bytes"]}
                       for r in rows}}
    lines += ["", "Machine-readable record:", "", "```json", json.dumps(rec), "```"]
    open(args.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
