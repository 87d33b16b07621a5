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
        e = EtdRdp(ins["shape"], ins["bcs"], ins["D"], ens.k, ens.model, ins["params"])
        u = torch.from_numpy(ens.states[i].copy()).cuda()
        e.step(u, 3)
        torch.cuda.synchronize()
        single = u.cpu().numpy()
        assert np.abs(got[i] - single).max() <= 1e-14 * np.abs(single).max(), i
        if i < 4:
            hs = [1.0 / (n - 1) if bc == "neumann" else 1.0 / n for n, bc in zip(ins["shape"], ins["bcs"])]
            ref = O.etd_rdp_if_run(ens.states[i], ens.k, ins["D"], ins["bcs"], hs, ens.model, ins["params"], 3)
            assert np.linalg.norm(got[i] - ref) / np.linalg.norm(ref) < 1e-12, i


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
