"""Throughput benchmark of the ETD-RDP-IF step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                [--no-cpu-baseline] [--pass-steps P]

A "step" is one full ETD-RDP-IF time step (all passes) over the workload's
state, which is resident in HBM before timing starts.  Prints one JSON line.

* value        cell-species-steps per second over the K timed steps
               (HIP events on the stream the kernels run on).
* roofline     the dominant kernel (the pass with the largest average
               launch time, timed with HIP events over P launches of that
               pass alone) against 8 TB/s HBM: achieved = algorithmic bytes
               of one launch / its average duration.  Algorithmic bytes per
               cell-species: pass 1 reads U and writes c1, c2, w (4 words),
               a middle pass reads and writes all three (6 words), the last
               pass reads three and writes U (4 words); 1 word = 8 bytes
               (4 with --precision f32, 16 for a complex species).
               step_effective_GBps is the same ratio for the whole step;
               traffic (counter-measured HBM bytes per launch, when stored
               for these kernel sources) gives traffic_GBps beside it.
* cpu_baseline the FP64 oracle on the host's cores, on a bounded sample of
               the same workload (stated in "sample"): "value" with its line
               solves spread over a process pool ("cores" processes; each
               pass's lines are cut into blocks along another axis and each
               block is solved by the oracle's own routine), and
               "single_thread" with everything on one thread.  Host CPU
               model, thread count and memory are recorded beside it.  It
               runs before the GPU is touched.
* ceiling      the same device's rate for plain streaming kernels (copy,
               read-only, write-only sweeps of 2 GiB, HIP events), so the
               passes can be read against what simple code reaches here;
               each pass also reports its rate as a fraction of the copy.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def pass_words(d: int):
    """Algorithmic FP64 words per cell-species moved by each pass."""
    return [4] + [6] * (d - 2) + [4]


def pass_names(e, d: int):
    """Kernel names (as rocprofv3 prints them, shortened) of each pass."""
    return [e.pass_kernel(p) for p in range(1, d + 1)]


def host_info():
    """CPU model, hardware threads and memory of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ram = os.sysconf("SC_PAGE_SIZE") * os.sysconf("SC_PHYS_PAGES") / 2**30
    except (ValueError, OSError):
        ram = None
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": aff,
            "ram_GiB": round(ram, 1) if ram else None}


def pool_size():
    """Worker processes for the all-core oracle timing: the CPUs this process
    may use, at most 16 (the host's share per GPU)."""
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, aff))


# Shared state of the all-core oracle timing: the oracle's own line-solve
# routines and two shared byte buffers, set before the pool forks.
_POOL = {}


def _pool_init():
    from threadpoolctl import threadpool_limits
    _POOL["limits"] = threadpool_limits(limits=1)


def _pool_task(args):
    import numpy as np
    fname, shape, dtype, sax, lo, hi, fargs = args
    inb, outb = _POOL["bufs"]
    cnt = int(np.prod(shape))
    X = np.frombuffer(inb, dtype=dtype, count=cnt).reshape(shape)
    Y = np.frombuffer(outb, dtype=dtype, count=cnt).reshape(shape)
    sl = [slice(None)] * len(shape)
    sl[sax] = slice(lo, hi)
    Y[tuple(sl)] = _POOL["orig"][fname](X[tuple(sl)], *fargs)
    return 0


class OraclePool:
    """Runs the oracle's per-axis line routines (solve_axis, solve_axis_T,
    laplacian_axis) over a process pool: every line of a pass is independent,
    so the array is cut into blocks along another axis and the oracle's own
    routine handles each block in a worker.  Arrays travel through shared
    memory.  Inside ``with pool:`` the oracle module calls the pooled
    versions; its arithmetic is unchanged."""

    FUNCS = ("solve_axis", "solve_axis_T", "laplacian_axis")

    def __init__(self, nproc: int, max_bytes: int):
        import multiprocessing as mp

        import oracle.etd_rdp_oracle as OM
        ctx = mp.get_context("fork")
        _POOL["bufs"] = (ctx.RawArray("b", max_bytes), ctx.RawArray("b", max_bytes))
        _POOL["orig"] = {f: getattr(OM, f) for f in self.FUNCS}
        self.OM, self.n, self.max_bytes = OM, nproc, max_bytes
        self.pool = ctx.Pool(nproc, initializer=_pool_init)

    def _pooled(self, fname):
        import numpy as np
        orig = _POOL["orig"][fname]

        def run(U, axis, *rest):
            U = np.asarray(U)
            coefs_complex = fname != "laplacian_axis" and np.iscomplexobj(rest[0])
            if U.nbytes > self.max_bytes or (coefs_complex and not np.iscomplexobj(U)):
                return orig(U, axis, *rest)
            npax = U.ndim - axis  # numpy axis of spatial axis `axis`
            # blocks along another spatial axis (never the species axis: each
            # species has its own coefficient)
            others = [a for a in range(1, U.ndim) if a != npax]
            if not others:
                return orig(U, axis, *rest)
            sax = max(others, key=lambda a: U.shape[a])
            inb, outb = _POOL["bufs"]
            X = np.frombuffer(inb, dtype=U.dtype, count=U.size).reshape(U.shape)
            X[...] = U
            cuts = np.linspace(0, U.shape[sax], min(self.n, U.shape[sax]) + 1).astype(int)
            tasks = [(fname, U.shape, U.dtype.str, sax, int(lo), int(hi), (axis,) + tuple(rest))
                     for lo, hi in zip(cuts[:-1], cuts[1:]) if hi > lo]
            self.pool.map(_pool_task, tasks)
            return np.frombuffer(outb, dtype=U.dtype, count=U.size).reshape(U.shape).copy()
        return run

    def __enter__(self):
        for f in self.FUNCS:
            setattr(self.OM, f, self._pooled(f))
        return self

    def __exit__(self, *exc):
        for f in self.FUNCS:
            setattr(self.OM, f, _POOL["orig"][f])
        return False

    def close(self):
        self.pool.terminate()
        self.pool.join()


def _time_loop(step, budget_s, max_steps=1000):
    steps, t0 = 0, time.perf_counter()
    while True:
        step()
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= max_steps:
            return steps, el


def cpu_baseline(name: str, budget_s: float = 10.0):
    """Time the oracle on a reduced grid of the same workload: all cores
    (line solves over a process pool) and one thread, about budget_s seconds
    of work each."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle as O
    from paper_2001_11220_amd import workloads as W

    sample_n = {"grayscott3d": 64, "schnakenberg3d": 64, "brusselator2d": 64,
                "schnakenberg3d_adjoint": 64, "cgl3d_complex": 64, "cgl2d_complex": 400,
                "grayscott4d": 16, "grayscott5d": 8}[name]
    prob = W.WORKLOADS[name](n=sample_n)
    cs = prob.cells * prob.s
    state = {"u": prob.initial()}

    def one():
        state["u"] = O.etd_rdp_if_step(state["u"], prob.k, prob.D, prob.bcs, prob.hs(), prob.model,
                                       prob.oracle_params())

    ncores = pool_size()
    pool = OraclePool(ncores, state["u"].nbytes)
    try:
        with threadpool_limits(limits=1), pool:
            one()  # untimed: the workers' first touch of the shared buffers
            state["u"] = prob.initial()
            steps_p, el_p = _time_loop(one, budget_s)
    finally:
        pool.close()
    state["u"] = prob.initial()
    with threadpool_limits(limits=1):
        steps_1, el_1 = _time_loop(one, budget_s)
    shape = "x".join(map(str, prob.shape))
    return {"value": cs * steps_p / el_p, "unit": "cell-species-steps/s", "cores": ncores,
            "kind": "oracle",
            "sample": f"{name} at {shape} (same coefficients and initial-data recipe), {steps_p} "
                      f"steps in {el_p:.1f} s, line solves over {ncores} processes",
            "single_thread": {"value": cs * steps_1 / el_1, "cores": 1,
                              "sample": f"{name} at {shape}, {steps_1} steps in {el_1:.1f} s, 1 thread"},
            "host": host_info()}


def ceiling(dev, nbytes: int = 1 << 31, reps: int = 10):
    """Device rate of plain streaming kernels over nbytes (copy, read-only,
    write-only), in GB/s of bytes moved; HIP events on the current stream."""
    import torch

    from paper_2001_11220_amd.etd import calib_stream

    x = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    sink = torch.zeros(8, dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream()
    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    out = {"bytes": nbytes, "how": f"etd_calib_stream sweeps of {nbytes / 2**30:.0f} GiB "
                                   "(256-thread blocks, four 16-byte accesses in flight per thread; "
                                   "copy and write with plain and with non-temporal stores; a copy "
                                   "with 1024-thread blocks streaming contiguous ranges) and "
                                   "torch's device copy; best over block counts and store kinds, "
                                   "HIP events"}
    variants = {"copy": ("copy", "copy_nt", "copy_ranges"), "read": ("read",),
                "write": ("write", "write_nt")}
    for kind, moved in (("copy", 2 * nbytes), ("read", nbytes), ("write", nbytes)):
        best, best_v = 0.0, None
        for var in variants[kind]:
            for blocks in ((ncu * 2, ncu * 4, ncu * 8) if var == "copy_ranges" else (ncu * 4, ncu * 8, ncu * 16)):
                src, dst = (x, y) if kind == "copy" else ((x, sink) if kind == "read" else (None, y))
                calib_stream(var, src, dst, nbytes, blocks)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(st)
                for _ in range(reps):
                    calib_stream(var, src, dst, nbytes, blocks)
                b.record(st)
                torch.cuda.synchronize()
                rate = moved * reps / (a.elapsed_time(b) / 1e3) / 1e9
                out[f"{var}_{blocks // ncu}x_GBps"] = rate
                if rate > best:
                    best, best_v = rate, var
        out[f"{kind}_GBps"] = best
        out[f"{kind}_variant"] = best_v
    y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        y.copy_(x)
    b.record(st)
    torch.cuda.synchronize()
    out["torch_copy_GBps"] = 2 * nbytes * reps / (a.elapsed_time(b) / 1e3) / 1e9
    del x, y, sink
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's step count)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="schnakenberg3d",
                    help="default: the 512^3 Dirichlet Schnakenberg system, the largest "
                         "single-problem configuration")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pass-steps", type=int, default=50)
    ap.add_argument("--checkpoint-every", type=int, default=20,
                    help="gradient workload: steps between stored states (checkpointed plan)")
    ap.add_argument("--keep", default="auto", choices=["auto", "true", "false"],
                    help="gradient workload: store every step's carried arrays (true), "
                         "checkpoint and recompute (false), or store when it fits (auto)")
    ap.add_argument("--n", type=int, default=None,
                    help="grid points per axis (default: the workload's own size)")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"],
                    help="arithmetic and storage type of the single-problem workloads")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-ceiling", action="store_true",
                    help="skip the streaming-kernel ceiling sweeps (profiler runs)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU design is described but not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2001_11220_amd import workloads as W
    from paper_2001_11220_amd.etd import EtdRdp

    if args.precision != "f64" and args.workload == "schnakenberg3d_adjoint":
        print(f"bench.py: workload {args.workload} runs in f64 only", file=sys.stderr)
        sys.exit(2)
    if args.workload not in W.WORKLOADS and args.workload != "brusselator_ensemble":
        print(f"bench.py: unknown workload {args.workload}", file=sys.stderr)
        sys.exit(2)
    if (args.precision != "f64" and args.workload in W.WORKLOADS
            and W.WORKLOADS[args.workload](n=8).is_complex):
        print(f"bench.py: workload {args.workload} runs in complex FP64 only", file=sys.stderr)
        sys.exit(2)
    # The oracle's timing runs first, before anything initialises the GPU
    # (its worker processes are forked from this one).
    cpu = None
    if not args.no_cpu_baseline:
        if args.workload == "brusselator_ensemble":
            cpu = cpu_baseline_ensemble()
        elif args.workload == "schnakenberg3d_adjoint":
            cpu = cpu_baseline_adjoint()
        else:
            cpu = cpu_baseline(args.workload)
        print(f"[bench] cpu baseline: {cpu['value']:.3e} {cpu['unit']} on {cpu['cores']} processes, "
              f"{cpu['single_thread']['value']:.3e} on one thread", file=sys.stderr, flush=True)
    if args.workload == "brusselator_ensemble":
        if args.steps is None:
            args.steps = 200
        return bench_ensemble(args, cpu)
    if args.workload == "schnakenberg3d_adjoint":
        return bench_adjoint(args, cpu)
    prob = W.WORKLOADS[args.workload](**({"n": args.n} if args.n else {}))
    if args.steps is None:
        args.steps = prob.nsteps
    prec = args.precision
    if prob.is_complex:
        if prec != "f64":
            print(f"bench.py: workload {args.workload} runs in complex FP64 only", file=sys.stderr)
            sys.exit(2)
        prec = "c128"
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    e = EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params, h=prob.h,
               shift=prob.shift, device=dev, precision=prec)
    esize = {"f64": 8, "f32": 4, "c128": 16}[prec]
    u = torch.from_numpy(prob.initial()).to(dev)
    if prec == "f32":
        u = u.float()
    e.workspace()
    stream = torch.cuda.current_stream()
    print(f"[bench] {prob.name} shape={prob.shape} bcs={prob.bcs} ws={e.ws_bytes/2**30:.2f} GiB",
          file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        e.step(u, 1)
    torch.cuda.synchronize()
    # The K timed steps are one launch of a HIP graph recorded (not run)
    # beforehand: no host launch overhead inside the timed region.
    e.use_graph(True)
    e.record_graph(u, args.steps)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    e.step(u, args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    e.use_graph(False)
    ms_step = ms / max(args.steps, 1)
    cs = prob.cells * prob.s
    value = cs * args.steps / (ms / 1e3)
    finite = bool(torch.isfinite(u).all().item())
    print(f"[bench] {args.steps} steps in {ms:.2f} ms ({ms_step:.4f} ms/step), finite={finite}",
          file=sys.stderr, flush=True)

    # Per-pass kernel timing (each pass alone, same arrays as in a step).
    d = len(prob.shape)
    words = pass_words(d)
    names = pass_names(e, d)
    per = []
    for p in range(1, d + 1):
        e.run_pass(u, p)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.pass_steps):
            e.run_pass(u, p)
        b.record(stream)
        torch.cuda.synchronize()
        t_ms = a.elapsed_time(b) / args.pass_steps
        byts = words[p - 1] * esize * cs
        per.append({"pass": p, "kernel": names[p - 1], "avg_ms": t_ms, "alg_bytes": byts,
                    "GBps": byts / (t_ms / 1e3) / 1e9})
        print(f"[bench] pass {p} ({names[p-1]}): {t_ms*1e3:.1f} us/launch, "
              f"{per[-1]['GBps']:.0f} GB/s algorithmic", file=sys.stderr, flush=True)
    ceil = None
    if not args.no_ceiling:
        ceil = ceiling(dev)
        for r in per:
            r["frac_of_copy"] = r["GBps"] / ceil["copy_GBps"]
        print(f"[bench] ceiling: copy {ceil['copy_GBps']:.0f}, read {ceil['read_GBps']:.0f}, "
              f"write {ceil['write_GBps']:.0f}, torch copy {ceil['torch_copy_GBps']:.0f} GB/s",
              file=sys.stderr, flush=True)
    dom = max(per, key=lambda r: r["avg_ms"])
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        from paper_2001_11220_amd.profiling import kernel_rev
        tr = json.load(open(TRAFFIC_FILE)).get(prob.name, {})
        rec = tr.get("kernels", {}).get(dom["kernel"])
        if rec and tr.get("kernel_rev") == kernel_rev():
            traffic = rec["bytes_per_launch"]
    if args.calib_copy:
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    step_bytes = sum(words) * esize * cs
    roof = {"bound": "hbm", "achieved": dom["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dom["GBps"] / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom["kernel"],
            "pass": dom["pass"], "avg_launch_us": dom["avg_ms"] * 1e3,
            "alg_bytes_per_launch": dom["alg_bytes"],
            "step_effective_GBps": step_bytes / (ms_step / 1e3) / 1e9,
            "step_frac": step_bytes / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
            "passes": [{k: r[k] for k in ("pass", "kernel", "avg_ms", "GBps", "frac_of_copy") if k in r}
                       for r in per]}
    if traffic is not None:
        # counted HBM bytes of the dominant kernel per second of its launch time
        roof["traffic_GBps"] = traffic / (dom["avg_ms"] / 1e3) / 1e9
        roof["traffic_frac"] = roof["traffic_GBps"] / HBM_PEAK_GBS

    out = {
        "metric": "cell-species-steps/sec",
        "value": value,
        "unit": "cell-species-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic (seeded initial data, no dataset)",
        "config": {"workload": prob.name, "grid": list(prob.shape), "bcs": list(prob.bcs),
                   "species": prob.s, "k": prob.k, "model": prob.model,
                   "launch": f"the {args.steps} timed steps as one HIP graph launch",
                   "state_finite": finite},
        "roofline": roof,
        "ceiling": ceil,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline_ensemble(budget_s: float = 10.0):
    """The oracle stepping instances of the ensemble (in draw order, one step
    each, cycling): all cores (instances spread over a process pool) and one
    thread."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    from paper_2001_11220_amd import workloads as W

    ens = W.brusselator_ensemble()
    ncores = pool_size()
    ctx = mp.get_context("fork")
    _POOL["ens"] = ens
    per_round = 4 * ncores  # instances per pool round
    with ctx.Pool(ncores, initializer=_pool_init) as pool:
        done, cells, t0 = 0, 0, time.perf_counter()
        while True:
            idx = [(done + j) % len(ens.instances) for j in range(per_round)]
            cells += sum(pool.map(_ens_step, idx))
            done += per_round
            el = time.perf_counter() - t0
            if el >= budget_s:
                break
    with threadpool_limits(limits=1):
        done1, cells1, t1 = 0, 0, time.perf_counter()
        while True:
            cells1 += _ens_step(done1 % len(ens.instances))
            done1 += 1
            el1 = time.perf_counter() - t1
            if el1 >= budget_s:
                break
    return {"value": cells / el, "unit": "cell-species-steps/s", "cores": ncores, "kind": "oracle",
            "sample": f"brusselator_ensemble: {done} instance-steps (instances in draw order, one "
                      f"step each) in {el:.1f} s over {ncores} processes",
            "single_thread": {"value": cells1 / el1, "cores": 1,
                              "sample": f"{done1} instance-steps in {el1:.1f} s, 1 thread"},
            "host": host_info()}


def _ens_step(i):
    """One oracle step of ensemble instance i; returns its cell-species."""
    import oracle as O
    ens = _POOL["ens"]
    ins, u = ens.instances[i], ens.states[i]
    hs = [1.0 / (n - 1) if b == "neumann" else 1.0 / n for n, b in zip(ins["shape"], ins["bcs"])]
    O.etd_rdp_if_step(u, ens.k, ins["D"], ins["bcs"], hs, ens.model, ins["params"])
    return u.size


def bench_ensemble(args, cpu=None):
    """1024 independent 2-D Brusselators of uneven size, all steps recorded in
    one HIP graph; reported against the plain 2-D solver at N = 512 (both in
    --precision)."""
    import numpy as np
    import torch

    from paper_2001_11220_amd import workloads as W
    from paper_2001_11220_amd.etd import EtdRdp, EtdRdpBatch

    ens = W.brusselator_ensemble()
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    prec = args.precision
    wb = 4 if prec == "f32" else 8  # bytes per word
    b = EtdRdpBatch(ens.instances, ens.s, ens.model, ens.k, device=dev, precision=prec)
    stream = torch.cuda.current_stream()
    steps = args.steps
    print(f"[bench] ensemble of {b.n} instances in {len(b.groups())} groups, {ens.cell_species:.3e} "
          f"cell-species, {b.launches_per_step} launches/step, ws={b.ws_bytes/2**30:.2f} GiB",
          file=sys.stderr, flush=True)

    def graph_run():
        u = b.pack(ens.states)
        b.step(u, steps, use_graph=True)  # records the graph (untimed warm-up of `steps` steps)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        b.step(u, steps, use_graph=True)  # one graph launch
        ev1.record(stream)
        torch.cuda.synchronize()
        return u, ev0.elapsed_time(ev1)

    default_plan = b.plan
    _, ms_default = graph_run()
    # the autotuner (on a scratch copy of the state), then the timed run
    times = b.tune(b.pack(ens.states), reps=3)
    tuned_plan = b.plan
    u, ms = graph_run()
    ms_step = ms / steps
    print(f"[bench] default plan {ms_default / steps * 1e3:.1f} us/step, tuned plan {ms_step * 1e3:.1f} "
          f"us/step", file=sys.stderr, flush=True)
    for g, (n1, n2, cnt) in enumerate(b.groups()):
        print(f"[bench]   group {n1}x{n2} ({cnt}): pass 1 {times[g][0]} ms, pass 2 {times[g][1]} ms -> "
              f"forms {tuned_plan[2 * g]}, {tuned_plan[2 * g + 1]}", file=sys.stderr, flush=True)
    value = ens.cell_species * steps / (ms / 1e3)
    finite = bool(torch.isfinite(u).all().item())
    # plain 2-D solver at the largest instance size, same coefficients range
    p = EtdRdp((512, 512), ("neumann", "periodic"), (0.02, 0.02), ens.k, ens.model,
               {"a": 1.0, "b": 3.0}, device=dev, precision=prec)
    up = torch.from_numpy(np.stack([0.5 + 0.1 * np.random.default_rng(1).random((512, 512))
                                    for _ in range(2)])).to(dev, b.dtype)
    p.step(up, 20)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    p.step(up, steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    plain_ms = ev0.elapsed_time(ev1) / steps
    plain_value = 2 * 512 * 512 / (plain_ms / 1e3)
    print(f"[bench] ensemble {ms_step*1e3:.1f} us/step; plain 512^2 {plain_ms*1e3:.1f} us/step",
          file=sys.stderr, flush=True)
    eff = 8 * wb * value / 1e9  # 2-D: 8 words per cell-species-step
    out = {
        "metric": "cell-species-steps/sec",
        "value": value,
        "unit": "cell-species-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": steps,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic (seeded instance parameters and initial data, no dataset)",
        "config": {"workload": "brusselator_ensemble", "instances": b.n,
                   "cell_species": ens.cell_species, "launches_per_step": b.launches_per_step,
                   "graph": "all steps in one HIP graph launch", "state_finite": finite,
                   "groups": [list(g) for g in b.groups()],
                   "plan": "autotuned (etd_rdp_batch_tune), forms per (group, pass): "
                           + ",".join(map(str, tuned_plan)),
                   "default_plan_ms_per_step": ms_default / steps,
                   "default_plan": ",".join(map(str, default_plan)),
                   "tune_times_ms": times},
        "roofline": {"bound": "hbm", "achieved": eff, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": eff / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole step (all groups, 2 passes)",
                     "alg_bytes_per_step": 8 * wb * ens.cell_species},
        "plain_2d_512": {"value": plain_value, "ms_per_step": plain_ms,
                         "effective_GBps": 8 * wb * plain_value / 1e9},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline_adjoint(budget_s: float = 10.0):
    """The oracle's forward step plus reverse step on a 64^3 sample of the
    gradient workload: all cores (line routines over a process pool) and one
    thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle as O
    from paper_2001_11220_amd import workloads as W

    prob = W.schnakenberg3d_adjoint(n=64)
    cs = prob.cells * prob.s
    state = {}

    def reset():
        state["u"] = prob.initial()
        state["lam"] = np.random.default_rng(1).standard_normal(state["u"].shape)

    def one():
        u, lam = state["u"], state["lam"]
        un = O.etd_rdp_if_step(u, prob.k, prob.D, prob.bcs, prob.hs(), prob.model,
                               prob.oracle_params())
        state["lam"], _, _ = O.adjoint_step(u, lam, prob.k, prob.D, prob.bcs, prob.hs(), prob.model,
                                            prob.oracle_params())
        state["u"] = un

    reset()
    ncores = pool_size()
    pool = OraclePool(ncores, state["u"].nbytes)
    try:
        with threadpool_limits(limits=1), pool:
            one()  # untimed: the workers' first touch of the shared buffers
            reset()
            steps_p, el_p = _time_loop(one, budget_s)
    finally:
        pool.close()
    reset()
    with threadpool_limits(limits=1):
        steps_1, el_1 = _time_loop(one, budget_s)
    return {"value": cs * steps_p / el_p, "unit": "cell-species-steps/s", "cores": ncores,
            "kind": "oracle",
            "sample": f"schnakenberg3d_adjoint at 64x64x64: {steps_p} forward + reverse step pairs "
                      f"in {el_p:.1f} s, line routines over {ncores} processes",
            "single_thread": {"value": cs * steps_1 / el_1, "cores": 1,
                              "sample": f"{steps_1} forward + reverse step pairs in {el_1:.1f} s, "
                                        "1 thread"},
            "host": host_info()}


def bench_adjoint(args, cpu=None):
    """Gradient of a trajectory loss with respect to the initial state, D and
    the reaction parameters: 128^3 Neumann Schnakenberg, 400 steps, loss =
    sum (U(T) - U_target)^2 with U_target from (Du, Dv, a, b) perturbed by up
    to 5%.  Memory plan (--keep): every step's carried arrays stored when
    they fit in half the free device memory (then the checkpointed plan,
    checkpoints every m steps, is timed as well), else checkpoints every m
    steps.  value counts the cell-species-steps of the trajectory per second
    of forward + backward in the chosen plan."""
    import numpy as np
    import torch

    from paper_2001_11220_amd import workloads as W
    from paper_2001_11220_amd.adjoint import trajectory
    from paper_2001_11220_amd.etd import EtdRdp

    prob = W.schnakenberg3d_adjoint(**({"n": args.n} if args.n else {}))
    steps = args.steps if args.steps is not None else prob.nsteps
    every = args.checkpoint_every
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    e = EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params, h=prob.h,
               shift=prob.shift, device=dev)
    u0 = torch.from_numpy(prob.initial()).to(dev)
    D_t, th_t = W.gradient_target(prob)
    et = EtdRdp(prob.shape, prob.bcs, D_t, prob.k, prob.model, th_t, h=prob.h, shift=prob.shift,
                device=dev)
    target = u0.clone()
    et.step(target, steps)
    et.close()
    e.workspace(e.adj_ws_bytes)
    stream = torch.cuda.current_stream()
    cs = prob.cells * prob.s
    print(f"[bench] {prob.name} shape={prob.shape} steps={steps} checkpoint every {every}, "
          f"ws={e.adj_ws_bytes/2**30:.2f} GiB", file=sys.stderr, flush=True)

    keep = {"auto": "auto", "true": True, "false": False}[args.keep]
    if keep == "auto":
        free, _ = torch.cuda.mem_get_info(dev)
        keep = steps * (e.keep_bytes + u0.numel() * 8) <= 0.5 * free
    plan = "stored" if keep else "checkpointed"
    print(f"[bench] memory plan: {plan} ({steps} x {e.keep_bytes/2**20:.0f} MiB kept arrays)"
          if keep else f"[bench] memory plan: {plan}", file=sys.stderr, flush=True)

    def grad_run(nsteps, plan_keep):
        x = u0.clone().requires_grad_(True)
        p = torch.tensor(e.param_vector(), dtype=torch.float64, requires_grad=True)
        uT = trajectory(e, x, nsteps, p, checkpoint_every=every, keep=plan_keep)
        loss = ((uT - target) ** 2).sum()
        loss.backward()
        return loss, x.grad, p.grad

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed_grad(plan_keep):
        grad_run(min(args.warmup, steps), plan_keep)
        torch.cuda.synchronize()
        ev0.record(stream)
        out = grad_run(steps, plan_keep)
        ev1.record(stream)
        torch.cuda.synchronize()
        return out, ev0.elapsed_time(ev1)

    (loss, gx, gp), ms = timed_grad(keep)
    finite = bool(torch.isfinite(gx).all().item()) and bool(torch.isfinite(gp).all().item())
    other_ms = None
    if keep:
        # the checkpointed plan as well (checkpoints every `every` steps);
        # its gradient is bitwise the stored plan's
        (_, gx2, gp2), other_ms = timed_grad(False)
        same = bool(torch.equal(gx, gx2)) and bool(torch.equal(gp, gp2))
        print(f"[bench] checkpointed plan: {other_ms:.1f} ms, gradient bitwise equal to the stored "
              f"plan's: {same}", file=sys.stderr, flush=True)
        del gx2, gp2
        torch.cuda.empty_cache()
    # plain forward of the same trajectory
    u = u0.clone()
    e.step(u, 10)
    torch.cuda.synchronize()
    ev0.record(stream)
    e.step(u, steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    fwd_ms = ev0.elapsed_time(ev1)
    # one reverse step alone, repeated
    lam = torch.randn_like(u0)
    g = torch.zeros(e.grad_size, dtype=torch.float64, device=dev)
    e.adjoint(u0, lam, lam_out=lam, grad=g)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.pass_steps):
        e.adjoint(u0, lam, lam_out=lam, grad=g)
    ev1.record(stream)
    torch.cuda.synchronize()
    adj_ms = ev0.elapsed_time(ev1) / args.pass_steps
    if args.calib_copy:
        # one plain 1 GiB device copy (scale of the counter readings)
        xc = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        yc = torch.empty_like(xc)
        yc.copy_(xc)
        torch.cuda.synchronize()
        del xc, yc
    # the reverse step on kept arrays (what the stored plan runs)
    kept = e.new_keep(1)
    e.step_keep(u0.clone(), kept[0])
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.pass_steps):
        e.adjoint(u0, lam, lam_out=lam, grad=g, kept=kept[0])
    ev1.record(stream)
    torch.cuda.synchronize()
    kept_ms = ev0.elapsed_time(ev1) / args.pass_steps
    del kept
    value = cs * steps / (ms / 1e3)
    # Reverse step: forward recompute of passes 1-2 (4 + 6 words), reverse
    # passes for axis 3 (7), axis 2 (9) and axis 1 (5): 31 words per
    # cell-species; 21 on kept arrays (the three reverse passes).
    adj_bytes = 31 * 8 * cs
    adj_gbs = adj_bytes / (adj_ms / 1e3) / 1e9
    kept_bytes = 21 * 8 * cs
    kept_gbs = kept_bytes / (kept_ms / 1e3) / 1e9
    print(f"[bench] gradient {ms:.1f} ms ({ms/steps:.3f} ms/step); forward alone {fwd_ms:.1f} ms; "
          f"reverse step {adj_ms*1e3:.1f} us ({adj_gbs:.0f} GB/s algorithmic), on kept arrays "
          f"{kept_ms*1e3:.1f} us ({kept_gbs:.0f} GB/s); loss={float(loss.detach()):.6e}",
          file=sys.stderr, flush=True)
    if keep:
        roof = {"bound": "hbm", "achieved": kept_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": kept_gbs / HBM_PEAK_GBS, "traffic": None,
                "kernel": "etd_rdp_adjoint_kept (one reverse step on kept arrays: 3 reverse passes)",
                "avg_launch_us": kept_ms * 1e3, "alg_bytes_per_launch": kept_bytes}
    else:
        roof = {"bound": "hbm", "achieved": adj_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": adj_gbs / HBM_PEAK_GBS, "traffic": None,
                "kernel": "etd_rdp_adjoint (one reverse step: 2 forward + 3 reverse passes)",
                "avg_launch_us": adj_ms * 1e3, "alg_bytes_per_launch": adj_bytes}
    out = {
        "metric": "cell-species-steps/sec",
        "value": value,
        "unit": "cell-species-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": min(args.warmup, steps),
        "ms_per_step": ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded initial data and target, no dataset)",
        "config": {"workload": prob.name, "grid": list(prob.shape), "bcs": list(prob.bcs),
                   "species": prob.s, "k": prob.k, "model": prob.model,
                   "gradient": "dL/d(u0, D, a, b, gamma) of sum (U(T) - U_target)^2",
                   "memory_plan": plan, "checkpoint_every": None if keep else every,
                   "grad_finite": finite, "forward_only_ms": fwd_ms,
                   "gradient_over_forward": ms / fwd_ms,
                   "checkpointed_ms": ms if not keep else other_ms,
                   "checkpointed_over_forward": (ms if not keep else other_ms) / fwd_ms,
                   "reverse_step_us": adj_ms * 1e3, "reverse_step_kept_us": kept_ms * 1e3},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
