"""GPU parity of the 4-D frame (the general-d form of Section 6: four split
factors per chain, axes 2 and 3 through middle passes) against the FP64
oracle.  Tolerances as in 3-D: rel-L2 <= 1e-12 after one step, <= 1e-10
after 20 steps; FP32 as in the FP32 tests."""

import numpy as np
import pytest

import oracle as O
from paper_2001_11220_amd import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _etd():
    from paper_2001_11220_amd import etd
    return etd


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def P(shape, bcs, D=(0.02, 0.011), k=0.05, model="brusselator", params=None, ic="uniform_noise"):
    params = params if params is not None else {"a": 1.0, "b": 3.4}
    return W.Problem("t4", tuple(shape), tuple(bcs), tuple(D), k, model, params, 1, seed=0, ic=ic,
                     ic_args={"base": 0.5, "amp": 0.3})


GS = {"F": 0.04, "kappa": 0.06}
CASES = [
    (P((12, 10, 8, 6), ("neumann", "periodic", "dirichlet", "neumann")), "auto"),
    (P((24, 16, 20, 9), ("periodic",) * 4, model="gray_scott", params=GS, D=(2e-5, 1e-5), k=1.0,
       ic="cube_patch"), "auto"),
    (P((96, 8, 70, 5), ("neumann", "periodic", "dirichlet", "neumann")), "auto"),  # chunk length 2
    (P((5, 3, 4, 130), ("dirichlet", "neumann", "periodic", "periodic")), "auto"),  # m = 3 on axis 4
    (P((3, 4, 192, 5), ("periodic", "neumann", "dirichlet", "neumann")), 2),  # axis 3 two lines per wave
    (P((160, 4, 3, 5), ("dirichlet", "periodic", "neumann", "dirichlet")), 2),  # axis 1 two lines per wave
    (P((7, 5, 6, 9), ("neumann",) * 4, model="enzyme", params={}, D=(0.2,)), "auto"),
]


def _make(prob, lpw="auto", precision="f64"):
    return _etd().EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params, h=prob.h,
                         lines_per_wave=lpw, precision=precision)


@pytest.mark.parametrize("prob,lpw", CASES, ids=lambda c: "x".join(map(str, c.shape)) if hasattr(c, "shape") else str(c))
def test_one_step_4d_matches_oracle(prob, lpw):
    torch = _torch()
    u0 = prob.initial()
    e = _make(prob, lpw)
    names = [e.pass_kernel(p) for p in range(1, 5)]
    u = torch.from_numpy(u0).cuda()
    e.step(u, 1)
    torch.cuda.synchronize()
    e.close()
    ref = O.etd_rdp_if_run(u0, prob.k, prob.D, prob.bcs, prob.hs(), prob.model, prob.oracle_params(), 1)
    err = rel_l2(u.cpu().numpy(), ref)
    print(f"[4-D one step] {prob.shape} {names} rel_l2={err:.2e}", flush=True)
    assert err <= 1e-12, err


def test_20_steps_4d_matches_oracle():
    torch = _torch()
    prob = P((20, 12, 9, 16), ("periodic", "neumann", "periodic", "dirichlet"))
    u0 = prob.initial()
    e = _make(prob)
    u = torch.from_numpy(u0).cuda()
    e.step(u, 20)
    torch.cuda.synchronize()
    e.close()
    ref = O.etd_rdp_if_run(u0, prob.k, prob.D, prob.bcs, prob.hs(), prob.model, prob.oracle_params(), 20)
    err = rel_l2(u.cpu().numpy(), ref)
    print(f"[4-D 20 steps] rel_l2={err:.2e}", flush=True)
    assert err <= 1e-10, err


def test_4d_pass_intermediates_match_oracle():
    """Each carried triple (passes 1-3) in the layout etd_rdp_workspace_layout
    states, against the oracle's chains."""
    torch = _torch()
    prob = P((12, 10, 8, 6), ("neumann", "periodic", "dirichlet", "periodic"))
    u0 = prob.initial()
    e = _make(prob)
    inter = O.step_intermediates(u0, prob.k, prob.D, prob.bcs, prob.hs(), prob.model, prob.oracle_params())
    u = torch.from_numpy(u0).cuda()
    for npass in (1, 2, 3):
        e.debug_passes(u.clone(), npass)
        torch.cuda.synchronize()
        c1, c2, w = (x.cpu().numpy() for x in e.carried(npass))
        assert rel_l2(c1, inter[f"cU{npass}"]) <= 1e-12
        assert rel_l2(c2, inter[f"cf{npass}"]) <= 1e-12
        assert rel_l2(w, inter[f"y{npass}"]) <= 1e-12
    e.close()


def test_4d_f32_and_complex():
    torch = _torch()
    prob = P((24, 16, 20, 9), ("periodic", "neumann", "dirichlet", "periodic"))
    u0 = prob.initial()
    e = _make(prob, precision="f32")
    u = torch.from_numpy(u0).cuda().float()
    e.step(u, 1)
    torch.cuda.synchronize()
    e.close()
    ref = O.etd_rdp_if_run(u0, prob.k, prob.D, prob.bcs, prob.hs(), prob.model, prob.oracle_params(), 1)
    err32 = rel_l2(u.cpu().numpy().astype(np.float64), ref)
    z = W.Problem("z4", (20, 12, 10, 8), ("periodic", "neumann", "dirichlet", "periodic"), (1 + 0.5j,), 0.05,
                  "cgl_z", {"beta": 1.3}, 1, h=(1.0,) * 4, seed=0, ic="complex_noise", ic_args={"amp": 0.5})
    z0 = z.initial()
    ez = _etd().EtdRdp(z.shape, z.bcs, z.D, z.k, z.model, z.params, h=z.h, precision="c128")
    uz = torch.from_numpy(z0).cuda()
    ez.step(uz, 1)
    torch.cuda.synchronize()
    ez.close()
    refz = O.etd_rdp_if_run(z0, z.k, z.D, z.bcs, z.hs(), z.model, z.oracle_params(), 1)
    errz = rel_l2(uz.cpu().numpy(), refz)
    print(f"[4-D f32] rel_l2={err32:.2e}  [4-D complex] rel_l2={errz:.2e}", flush=True)
    assert err32 <= 1e-5 and errz <= 1e-12, (err32, errz)


def test_4d_schroedinger_with_field_matches_oracle():
    """The per-cell reaction field in 4-D (its copy in the last pass's layout
    reverses all four axes)."""
    torch = _torch()
    shape = (12, 7, 10, 9)
    z = W.Problem("z4f", shape, ("neumann", "periodic", "dirichlet", "neumann"), (1j,), 1e-3, "nls_z",
                  {"B": 0.4, "C": -1.0}, 1, seed=0, ic="complex_noise", ic_args={"amp": 0.5})
    z0 = z.initial()
    field = np.random.default_rng(5).standard_normal(shape[::-1])
    e = _etd().EtdRdp(z.shape, z.bcs, z.D, z.k, z.model, z.params, precision="c128", field=True)
    u = torch.from_numpy(z0).cuda()
    e.set_field(torch.from_numpy(field).cuda())
    e.step(u, 2)
    torch.cuda.synchronize()
    e.close()
    ref = O.etd_rdp_if_run(z0, z.k, z.D, z.bcs, z.hs(), z.model, dict(z.oracle_params(), Bfield=field), 2)
    err = rel_l2(u.cpu().numpy(), ref)
    print(f"[4-D complex field, 2 steps] rel_l2={err:.2e}", flush=True)
    assert err <= 1e-12, err
