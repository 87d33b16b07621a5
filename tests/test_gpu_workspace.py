"""A workspace whose contents were changed outside the library is refilled
after etd_rdp_forget_workspace / etd_rdp_batch_forget_workspace (the
library cannot tell a new buffer at an old address from the old one)."""

import numpy as np
import pytest

import oracle as O
from paper_2001_11220_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_forgotten_workspace_is_filled_again():
    import torch
    from paper_2001_11220_amd.etd import EtdRdp
    prob = W.grayscott3d(shape=(64, 24, 40))
    e = EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params)
    u0 = prob.initial()
    ref = O.etd_rdp_if_run(u0, prob.k, prob.D, prob.bcs, prob.hs(), prob.model, prob.params, 2)
    print(f"[workspace] {prob.name} {prob.shape}", flush=True)
    for _ in range(2):
        u = torch.from_numpy(u0).cuda()
        e.step(u, 2)
        torch.cuda.synchronize()
        err = float(np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref))
        assert err <= 1e-12, err
        e.workspace().fill_(0)  # the tables it held are gone
        e.forget_workspace()
    e.close()


def test_forgotten_ensemble_workspace_is_filled_again():
    import torch
    from paper_2001_11220_amd.etd import EtdRdpBatch
    ens = W.brusselator_ensemble(ninst=6, sizes=(64, 96, 128))
    b = EtdRdpBatch(ens.instances, ens.s, ens.model, ens.k)
    refs = []
    for ins, st in zip(ens.instances, ens.states):
        hs = [O.default_h(n, bc) for n, bc in zip(ins["shape"], ins["bcs"])]
        refs.append(O.etd_rdp_if_run(st, ens.k, ins["D"], ins["bcs"], hs, ens.model, ins["params"], 2))
    print(f"[workspace] ensemble of {b.n}", flush=True)
    for use_graph in (True, False, True):
        u = b.pack(ens.states)
        b.step(u, 2, use_graph=use_graph)
        torch.cuda.synchronize()
        for i, ref in enumerate(refs):
            got = b.view(u, i).cpu().numpy()
            assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-12, i
        b.workspace().fill_(0)
        b.forget_workspace()
    b.close()
