"""Graph mode of the single-problem step (etd_rdp_set_graph): replays of the
recorded graph equal direct launches bit for bit, with the program's own
eager work and synchronisations between replays; a new (u, nsteps) records
a new graph; results match the oracle."""

import numpy as np
import pytest

import oracle as O
from paper_2001_11220_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prob", [W.brusselator2d(n=64), W.grayscott3d(shape=(64, 40, 24)),
                                  W.grayscott4d(shape=(16, 12, 8, 6))],
                         ids=["2d", "3d", "4d"])
def test_graph_replays_equal_direct_launches(prob):
    import torch
    from paper_2001_11220_amd.etd import EtdRdp
    print(f"[graph] {prob.name} {prob.shape}", flush=True)
    e = EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params)
    u0 = torch.from_numpy(prob.initial()).cuda()
    ref = u0.clone()
    e.step(ref, 3)
    e.step(ref, 3)
    e.step(ref, 3)
    g = u0.clone()
    e.use_graph(True)
    for rep in range(3):  # record, then two replays of the same graph
        e.step(g, 3)
        torch.cuda.synchronize()
        _ = (g * 2.0).sum().item()  # eager work between replays
    assert torch.equal(g, ref)
    h = u0.clone()
    e.step(h, 2)  # another nsteps: a new graph
    e.step(h, 7)
    torch.cuda.synchronize()
    assert torch.equal(h, ref)
    e.close()
    got = g.cpu().numpy()
    want = O.etd_rdp_if_run(prob.initial(), prob.k, prob.D, prob.bcs, prob.hs(), prob.model, prob.params, 9)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-11


def test_recorded_graph_runs_only_when_stepped():
    import torch
    from paper_2001_11220_amd.etd import EtdRdp
    prob = W.brusselator2d(n=48)
    e = EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params)
    u0 = torch.from_numpy(prob.initial()).cuda()
    ref = u0.clone()
    e.step(ref, 4)
    u = u0.clone()
    e.use_graph(True)
    e.record_graph(u, 4)
    torch.cuda.synchronize()
    assert torch.equal(u, u0)  # recording runs nothing
    e.step(u, 4)
    torch.cuda.synchronize()
    assert torch.equal(u, ref)
    e.close()
