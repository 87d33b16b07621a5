"""Summaries of rocprofv3 output for the benchmark (kernel times, HBM traffic).

Usage (on result databases that rocprofv3 wrote):

  python -m paper_2001_11220_amd.profiling kernels RUN_results.db
  python -m paper_2001_11220_amd.profiling traffic --fetch F.db --write W.db \
      --copy-bytes B --workload NAME --out profiles/traffic.json

``traffic``: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of each of the
library's kernels, scaled by what the same counters read for the plain copy
kernel of ``B`` bytes that ``bench.py --calib-copy`` runs in the same process
(a copy of B bytes reads B and writes B bytes of HBM).
"""

from __future__ import annotations

import argparse
import collections
import hashlib
import json
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_rev() -> str:
    """Hash of the kernel sources; stored counter traffic is only valid for
    the revision it was measured on."""
    h = hashlib.sha1()
    for fn in ("etd_rdp.hip", "etd_general.hip", "etd_batch.hip", "etd_adjoint.hip", "etd_passes.hpp",
               "etd_device.hpp", "etd_launch.hpp", "etd_ctx.hpp", "etd_tables.hpp",
               "etd_tables.cpp"):
        with open(os.path.join(ROOT, "paper_2001_11220_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def short_name(name: str) -> str:
    n = name.split("(")[0]
    for pre in ("void ", "etd::"):
        n = n.replace(pre, "")
    return n.strip()


def kernel_times(db: str):
    """name -> list of durations (us) from a kernel-trace database."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end from kernels").fetchall()
    out = collections.defaultdict(list)
    for name, s, e in rows:
        out[name].append((e - s) / 1e3)
    return out


def counters(db: str):
    """(kernel name, counter) -> list of values per dispatch."""
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, counter_name, value from counters_collection").fetchall()
    out = collections.defaultdict(list)
    for kn, cn, v in rows:
        out[(kn, cn)].append(v)
    return out


def _copy_kernel(counts):
    """The calibration copy: the copy dispatch with the largest reading (the
    runtime's device-to-device blit kernel for torch's copy_)."""
    cands = [n for n in counts if "copy" in n.lower() and not n.startswith("void etd")]
    return max(cands, key=lambda n: max(counts[n])) if cands else None


def traffic(fetch_db: str, write_db: str, copy_bytes: int):
    fc, wc = counters(fetch_db), counters(write_db)
    fk = {k: v for (k, c), v in fc.items() if c == "FETCH_SIZE"}
    wk = {k: v for (k, c), v in wc.items() if c == "WRITE_SIZE"}
    copy_f, copy_w = _copy_kernel(fk), _copy_kernel(wk)
    if copy_f is None or copy_w is None:
        raise SystemExit("no calibration copy kernel in the counter runs (use bench.py --calib-copy)")
    # the calibration copy runs once; take its largest reading
    f_scale = copy_bytes / (max(fk[copy_f]) * 1024.0)
    w_scale = copy_bytes / (max(wk[copy_w]) * 1024.0)
    out = {"fetch_scale": f_scale, "write_scale": w_scale, "copy_kernel": short_name(copy_f),
           "kernels": {}}
    for name in fk:
        if not name.startswith("void etd::"):
            continue
        fv = sorted(fk[name])[len(fk[name]) // 2] * 1024.0 * f_scale
        wv = sorted(wk.get(name, [0.0]))[len(wk.get(name, [0.0])) // 2] * 1024.0 * w_scale
        out["kernels"][short_name(name)] = {"fetch_bytes": fv, "write_bytes": wv,
                                            "bytes_per_launch": fv + wv}
    return out


# SQ counters read by `sq`: wave-cycles resident, waiting (any reason, or
# for an instruction's dependency), and with an instruction of each kind in
# flight, per dispatch summed over the device.
SQ_COUNTERS = ("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY",
               "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_VMEM")


def sq_summary(db: str):
    """kernel -> {counter: median per dispatch} and the fractions of resident
    wave-cycles spent waiting / with VALU, LDS or VMEM instructions active."""
    cs = counters(db)
    out = {}
    for (kn, cn), v in cs.items():
        if not kn.startswith("void etd::") or cn not in SQ_COUNTERS:
            continue
        out.setdefault(short_name(kn), {})[cn] = sorted(v)[len(v) // 2]
    for k, r in out.items():
        wc = r.get("SQ_WAVE_CYCLES") or 0
        if wc:
            for cn, tag in (("SQ_WAIT_ANY", "wait_any"), ("SQ_WAIT_INST_ANY", "wait_inst"),
                            ("SQ_ACTIVE_INST_VALU", "valu"), ("SQ_ACTIVE_INST_LDS", "lds"),
                            ("SQ_ACTIVE_INST_VMEM", "vmem"), ("SQ_ACTIVE_INST_ANY", "any_inst")):
                if cn in r:
                    r[f"frac_{tag}"] = r[cn] / wc
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    q = sub.add_parser("sq")
    q.add_argument("db")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "sq":
        res = sq_summary(a.db)
        print(f"{'kernel':60s} {'waves':>8} {'wait':>6} {'inst':>6} {'valu':>6} {'lds':>6} {'vmem':>6}")
        for name, r in sorted(res.items()):
            print(f"{name[:60]:60s} {r.get('SQ_WAVES', 0):8.0f} {r.get('frac_wait_any', 0):6.2f} "
                  f"{r.get('frac_wait_inst', 0):6.2f} {r.get('frac_valu', 0):6.2f} "
                  f"{r.get('frac_lds', 0):6.2f} {r.get('frac_vmem', 0):6.2f}")
        return
    if a.cmd == "kernels":
        times = kernel_times(a.db)
        print(f"{'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10}  kernel")
        for name, v in sorted(times.items(), key=lambda kv: -sum(kv[1])):
            print(f"{len(v):6d} {sum(v)/len(v):10.1f} {min(v):10.1f} {max(v):10.1f}  {short_name(name)[:80]}")
        return
    res = traffic(a.fetch, a.write, a.copy_bytes)
    res["kernel_rev"] = kernel_rev()
    data = {}
    if os.path.exists(a.out):
        data = json.load(open(a.out))
    data[a.workload] = res
    with open(a.out, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    json.dump(res, sys.stdout, indent=1)
    print()


if __name__ == "__main__":
    main()
