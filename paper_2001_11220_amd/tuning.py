"""Autotuner front end: cached kernel plans.

The timing itself runs in the library (``etd_rdp_batch_tune`` times every
kernel form each ensemble group allows, pass by pass, and keeps the fastest).
This module keeps the winners in a JSON file so that a later run on the same
device, with the same kernel sources and the same problem layout, starts
from them without timing again:

    key = (device name, kernel source hash, precision, scheme, species,
           model, the groups' shapes and sizes)

``tune_batch(b, u)`` returns the plan it used; the cache file is
``$ETD_TUNE_CACHE`` or ``~/.cache/paper_2001_11220_amd/plans.json``.

``tune_lines_per_wave`` does the same for one problem: it times full steps
with one and with two lines per wavefront (where a line length allows two)
and returns the faster setting, which ``EtdRdp(lines_per_wave=...)`` takes.
"""

from __future__ import annotations

import hashlib
import json
import os
from typing import Optional

from . import profiling


def cache_path() -> str:
    return os.environ.get("ETD_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_2001_11220_amd", "plans.json")


def _device_name():
    import torch
    return torch.cuda.get_device_name(torch.cuda.current_device())


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, key, value):
    data = _load(path)
    data[key] = value
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def batch_key(b, scheme: str = "rdp") -> str:
    sig = {"device": _device_name(), "kernels": profiling.kernel_rev(), "precision": b.precision,
           "scheme": getattr(b, "scheme", scheme), "s": b.s, "model": getattr(b, "model", None),
           "groups": b.groups()}
    return "batch:" + hashlib.sha1(json.dumps(sig, sort_keys=True).encode()).hexdigest()[:20]


def tune_batch(b, u, reps: int = 3, path: Optional[str] = None, use_cache: bool = True):
    """Set b's plan from the cache, or run the autotuner on u (advancing it by
    one step) and store the result.  Returns (plan, times or None)."""
    path = path or cache_path()
    key = batch_key(b)
    if use_cache:
        hit = _load(path).get(key)
        if hit is not None:
            b.plan = hit["plan"]
            return b.plan, None
    times = b.tune(u, reps=reps)
    plan = b.plan
    if use_cache:
        _store(path, key, {"plan": plan, "times_ms": times})
    return plan, times


def tune_lines_per_wave(make, u0, steps: int = 5, path: Optional[str] = None, use_cache: bool = True,
                        key_extra=None):
    """make(lines_per_wave) -> EtdRdp.  Times `steps` steps from u0 with one
    and two lines per wavefront and returns the faster setting (1 or 2),
    cached like the ensemble plans."""
    import torch
    path = path or cache_path()
    e1 = make(1)
    sig = {"device": _device_name(), "kernels": profiling.kernel_rev(), "shape": list(e1.shape),
           "s": e1.s, "precision": e1.precision, "extra": key_extra}
    key = "lines:" + hashlib.sha1(json.dumps(sig, sort_keys=True).encode()).hexdigest()[:20]
    if use_cache:
        hit = _load(path).get(key)
        if hit is not None:
            e1.close()
            return hit["lines_per_wave"]
    cands = {1: e1}
    try:
        e2 = make(2)
        if any("32, 2" in e2.pass_kernel(p) for p in range(1, e2.d + 1)):
            cands[2] = e2
        else:
            e2.close()
    except Exception:  # no axis allows two lines per wavefront
        pass
    best, best_ms, times = 1, None, {}
    st = torch.cuda.current_stream()
    for lpw, e in cands.items():
        u = u0.clone()
        e.step(u, 1)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        e.step(u, steps)
        b.record(st)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        times[lpw] = ms
        if best_ms is None or ms < best_ms:
            best, best_ms = lpw, ms
    for e in cands.values():
        e.close()
    if use_cache:
        _store(path, key, {"lines_per_wave": best, "ms_per_step": times})
    return best
