"""The slab schedule of a 3-D step (passes 1 and 2 slab by slab along axis
3) gives the same result bit for bit as whole passes: it changes which
launch handles a line, not the arithmetic on it.  Checked for one and two
lines per wavefront, ragged last slabs, FP32 and a complex species, and
against the oracle."""

import numpy as np
import pytest

import oracle as O
from paper_2001_11220_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = [
    # shape (n_1, n_2, n_3), bcs, precision, lines per wave, slab planes
    ((64, 48, 40), ("periodic", "neumann", "dirichlet"), "f64", "auto", 16),
    ((64, 48, 40), ("periodic", "neumann", "dirichlet"), "f64", "auto", 7),   # ragged last slab
    ((96, 64, 96), ("neumann", "periodic", "dirichlet"), "f64", 2, 32),
    ((96, 64, 96), ("neumann", "periodic", "dirichlet"), "f64", 2, 40),       # 40 = 32 + 8
    ((40, 512, 24), ("dirichlet",) * 3, "f64", 1, 16),                        # chunks of 8 rows
    ((64, 48, 40), ("periodic", "neumann", "dirichlet"), "f32", "auto", 8),
    ((48, 40, 30), ("periodic",) * 3, "c128", "auto", 8),
]


@pytest.mark.parametrize("shape,bcs,prec,lpw,planes", CASES)
def test_slab_schedule_equals_whole_passes(shape, bcs, prec, lpw, planes):
    import torch
    from paper_2001_11220_amd import etd
    if prec == "c128":
        prob = W.cgl3d_complex(shape=shape)
        prob.bcs = bcs
        prob.h = None
    else:
        prob = W.grayscott3d(shape=shape)
        prob.bcs = bcs
    print(f"[slab] {shape} {bcs} {prec} lpw={lpw} planes={planes}", flush=True)
    e = etd.EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params,
                   lines_per_wave=lpw, precision=prec)
    u0 = prob.initial()
    dt = {"f64": torch.float64, "f32": torch.float32, "c128": torch.complex128}[prec]
    a = torch.from_numpy(u0).cuda().to(dt)
    b = a.clone()
    e.step(a, 2)
    e.slab = planes
    assert e.slab == planes
    e.step(b, 2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    ref = O.etd_rdp_if_run(u0, prob.k, prob.D, prob.bcs, prob.hs(), prob.model, prob.oracle_params(), 2)
    got = b.cpu().numpy().astype(np.complex128 if prec == "c128" else np.float64)
    tol = 1e-5 if prec == "f32" else 1e-12
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 2 * tol
    e.slab = 0
    e.close()


def test_slab_option_is_checked():
    from paper_2001_11220_amd import etd
    e = etd.EtdRdp((32, 32), ("neumann",) * 2, (0.1, 0.1), 0.1, "brusselator", {"a": 1.0, "b": 3.0})
    with pytest.raises(etd.EtdError):
        e.slab = 4  # 2-D: no slabs
    e.close()
    f = etd.EtdRdp((32, 24, 16), ("neumann",) * 3, (0.1, 0.1), 0.1, "brusselator", {"a": 1.0, "b": 3.0})
    f.slab = 16    # a whole axis 3: same as 0
    assert f.slab == 0
    with pytest.raises(etd.EtdError):
        f.slab = -1
    f.close()
