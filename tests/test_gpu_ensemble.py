"""Ensembles: every instance of a batch equals the single-problem GPU path
on that instance (same kernels' arithmetic, launched per instance), and the
oracle; graph replay equals direct launches."""

import numpy as np
import pytest

import oracle as O
from paper_2001_11220_amd import workloads as W

pytestmark = pytest.mark.gpu


def small_ensemble():
    return W.brusselator_ensemble(ninst=14, nsteps=5, seed=3,
                                  sizes=(3, 8, 17, 24, 40, 64, 96, 128, 160, 192, 288, 320))


def run_batch(ens, nsteps, use_graph=True):
    import torch
    from paper_2001_11220_amd.etd import EtdRdpBatch
    b = EtdRdpBatch(ens.instances, ens.s, ens.model, ens.k)
    u = b.pack(ens.states)
    b.step(u, nsteps, use_graph=use_graph)
    torch.cuda.synchronize()
    return [b.view(u, i).cpu().numpy() for i in range(b.n)], b


def test_ensemble_matches_single_problem_path_and_oracle():
    import torch
    from paper_2001_11220_amd.etd import EtdRdp
    ens = small_ensemble()
    got, b = run_batch(ens, 3)
    assert b.launches_per_step >= 2
    for i, ins in enumerate(ens.instances):
        # one line per wavefront: the chunking of the batch's default plan for
        # groups this small (the single path's automatic choice may take two
        # lines for passes of at most 128 lines, equal only to rounding)
        e = EtdRdp(ins["shape"], ins["bcs"], ins["D"], ens.k, ens.model, ins["params"], lines_per_wave=1)
        u = torch.from_numpy(ens.states[i].copy()).cuda()
        e.step(u, 3)
        torch.cuda.synchronize()
        single = u.cpu().numpy()
        assert np.abs(got[i] - single).max() <= 1e-14 * np.abs(single).max(), i
        hs = [1.0 / (n - 1) if bc == "neumann" else 1.0 / n for n, bc in zip(ins["shape"], ins["bcs"])]
        ref = O.etd_rdp_if_run(ens.states[i], ens.k, ins["D"], ins["bcs"], hs, ens.model, ins["params"], 3)
        assert np.linalg.norm(got[i] - ref) / np.linalg.norm(ref) < 1e-12, i
        assert np.abs(got[i] - ref).max() / np.abs(ref).max() < 1e-12, i


def test_graph_replay_equals_direct_launches():
    import torch
    from paper_2001_11220_amd.etd import EtdRdpBatch
    ens = small_ensemble()
    b = EtdRdpBatch(ens.instances, ens.s, ens.model, ens.k)
    u0 = b.pack(ens.states)
    a = u0.clone()
    b.step(a, 2, use_graph=False)
    b.step(a, 2, use_graph=False)
    g = u0.clone()
    b.step(g, 2, use_graph=True)   # captures
    torch.cuda.synchronize()
    b.step(g, 2, use_graph=True)   # replays (same u, ws, nsteps)
    torch.cuda.synchronize()
    assert torch.equal(a, g)


def test_f32_ensemble_matches_oracle_and_single_problem_f32_path():
    """FP32 ensemble (etd_rdp_batch_step_f32): every instance against the
    FP64 oracle within n times the single-problem FP32 tolerance (rel-L2
    1e-5 per step), and against the single-problem FP32 GPU path on that
    instance."""
    import torch
    from paper_2001_11220_amd.etd import EtdRdp, EtdRdpBatch
    ens = small_ensemble()
    nsteps = 3
    b = EtdRdpBatch(ens.instances, ens.s, ens.model, ens.k, precision="f32")
    u = b.pack(ens.states)
    assert u.dtype == torch.float32
    b.step(u, nsteps)
    torch.cuda.synchronize()
    worst = 0.0
    for i, ins in enumerate(ens.instances):
        got = b.view(u, i).cpu().numpy().astype(np.float64)
        hs = [1.0 / (n - 1) if bc == "neumann" else 1.0 / n for n, bc in zip(ins["shape"], ins["bcs"])]
        ref = O.etd_rdp_if_run(ens.states[i], ens.k, ins["D"], ins["bcs"], hs, ens.model, ins["params"], nsteps)
        tol = nsteps * 1e-5
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        worst = max(worst, err)
        assert err <= tol, (i, ins["shape"], err, tol)
        e = EtdRdp(ins["shape"], ins["bcs"], ins["D"], ens.k, ens.model, ins["params"], precision="f32",
                   lines_per_wave=1)  # the batch default plan's chunking, as above
        us = torch.from_numpy(ens.states[i].astype(np.float32)).cuda()
        e.step(us, nsteps)
        torch.cuda.synchronize()
        single = us.cpu().numpy().astype(np.float64)
        assert np.abs(got - single).max() <= 1e-5 * np.abs(single).max(), i
    print(f"[f32 ensemble] {b.n} instances, worst rel_l2={worst:.2e}", flush=True)
    # graph replay equals direct launches in FP32 too
    u0 = b.pack(ens.states)
    a, g = u0.clone(), u0.clone()
    b.step(a, 2, use_graph=False)
    b.step(g, 2, use_graph=True)
    torch.cuda.synchronize()
    assert torch.equal(a, g)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_etd1_ensemble_matches_oracle(prec):
    """The ensemble's first-order scheme (the ETD1 predictor alone, P_2 P_1
    (U + k F(U))): one step of every instance against the oracle's ETD1
    step (FP64: 1e-12; FP32: 1e-5)."""
    import torch
    from paper_2001_11220_amd.etd import EtdRdpBatch
    ens = small_ensemble()
    b = EtdRdpBatch(ens.instances, ens.s, ens.model, ens.k, scheme="etd1", precision=prec)
    u = b.pack(ens.states)
    b.step(u, 1)
    torch.cuda.synchronize()
    worst = 0.0
    for i, ins in enumerate(ens.instances):
        got = b.view(u, i).cpu().numpy().astype(np.float64)
        hs = [1.0 / (n - 1) if bc == "neumann" else 1.0 / n for n, bc in zip(ins["shape"], ins["bcs"])]
        ref = O.etd1_if_step(ens.states[i], ens.k, ins["D"], ins["bcs"], hs, ens.model, ins["params"])
        tol = 1e-12 if prec == "f64" else 1e-5
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        worst = max(worst, err)
        assert err <= tol, (i, ins["shape"], err, tol)
    print(f"[etd1 ensemble {prec}] {b.n} instances, worst rel_l2={worst:.2e}", flush=True)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_full_size_ensemble_one_step_sampled(prec):
    """The benchmark's ensemble (1024 instances, N = 64..512, recorded into a
    HIP graph as bench.py runs it, with the plan the autotuner picks on the
    device): one step, then the first and the last instance of every group
    (grid shape) and the last instance against the oracle (FP64: 1e-12;
    FP32: 1e-5)."""
    import torch
    from paper_2001_11220_amd.etd import EtdRdpBatch
    ens = W.brusselator_ensemble()
    b = EtdRdpBatch(ens.instances, ens.s, ens.model, ens.k, precision=prec)
    b.tune(b.pack(ens.states), reps=1)
    print(f"[full ensemble {prec}] tuned plan {b.plan}", flush=True)
    u = b.pack(ens.states)
    b.step(u, 1, use_graph=True)
    torch.cuda.synchronize()
    first_of, last_of = {}, {}
    for i, ins in enumerate(ens.instances):
        first_of.setdefault(tuple(ins["shape"]), i)
        last_of[tuple(ins["shape"])] = i
    sample = sorted(set(first_of.values()) | set(last_of.values()) | {b.n - 1})
    assert len(first_of) == 15 and b.launches_per_step == 30
    worst = 0.0
    for i in sample:
        ins = ens.instances[i]
        got = b.view(u, i).cpu().numpy().astype(np.float64)
        hs = [1.0 / (n - 1) if bc == "neumann" else 1.0 / n for n, bc in zip(ins["shape"], ins["bcs"])]
        ref = O.etd_rdp_if_step(ens.states[i], ens.k, ins["D"], ins["bcs"], hs, ens.model, ins["params"])
        tol = 1e-12 if prec == "f64" else 1e-5
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        worst = max(worst, err)
        assert err <= tol, (i, ins["shape"], err, tol)
    print(f"[full ensemble {prec}] {len(sample)} sampled instances, worst rel_l2={worst:.2e}", flush=True)
