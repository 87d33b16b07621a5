"""GPU parity of general line lengths: n with no split into at most 64 equal
chunks of at most 8 rows (79 and 361 of Sections 8.1 and 8.4, the timing
grids 799 and 801 of the enzyme and Brusselator tables, 1024 > 512, and
others), on every boundary condition and on every kind of pass (pass 1, a
middle pass of a 3-D and a 4-D step, the last pass, the single pass of a
1-D step), against the FP64 oracle.

Tolerances: FP64 and complex rel-L2 and largest pointwise error (relative to
the largest value) <= 1e-12 after one step; FP32 1e-5 per step."""

import numpy as np
import pytest

import oracle as O
from paper_2001_11220_amd import workloads as W

pytestmark = pytest.mark.gpu

GENERAL = [79, 361, 799, 801, 1024]
BCS = ["dirichlet", "neumann", "periodic"]
BRUSS = {"a": 1.0, "b": 3.4}


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def run(prob, u0, nsteps, scheme="rdp", precision="f64"):
    import torch
    from paper_2001_11220_amd import etd
    e = etd.EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params, h=prob.h,
                   scheme=scheme, precision=precision)
    names = [e.pass_kernel(p) for p in range(1, len(prob.shape) + 1)]
    splits = [e.line_split(a) for a in range(1, len(prob.shape) + 1)]
    u = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
    if precision == "f32":
        u = u.float()
    e.step(u, nsteps)
    torch.cuda.synchronize()
    e.close()
    got = u.cpu().numpy().astype(np.complex128 if precision == "c128" else np.float64)
    return got, names, splits


def check(prob, nsteps=1, scheme="rdp", precision="f64", tol=1e-12, u0=None):
    u0 = prob.initial() if u0 is None else u0
    got, names, splits = run(prob, u0, nsteps, scheme, precision)
    step = O.etd1_if_step if scheme == "etd1" else O.etd_rdp_if_step
    ref = u0
    for _ in range(nsteps):
        ref = step(ref, prob.k, prob.D, prob.bcs, prob.hs(), prob.model, prob.oracle_params())
    e2, em = rel_l2(got, ref), rel_max(got, ref)
    print(f"[general] {prob.shape} {prob.bcs} {prob.model} {precision} {scheme} {names} "
          f"rel_l2={e2:.2e} rel_max={em:.2e}", flush=True)
    assert e2 <= tol and em <= tol, (e2, em, tol)
    return names, splits


def general_split(n):
    m = -(-n // 64)
    return m, -(-n // m)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", GENERAL)
def test_general_line_on_every_pass(n, bc):
    """One step with the general axis as pass 1, the last pass (2-D), the
    middle pass (3-D), the third pass of a 4-D step and the one pass of a
    1-D step; the other axes regular."""
    other = {"dirichlet": "neumann", "neumann": "periodic", "periodic": "dirichlet"}[bc]
    cases = [
        ((n, 6), (bc, other), 0),
        ((5, n), (other, bc), 1),
        ((4, n, 3), (other, bc, "neumann"), 1),
        ((3, 4, n, 2), ("periodic", other, bc, "neumann"), 2),
        ((n,), (bc,), 0),
    ]
    for shape, bcs, ax in cases:
        prob = W.Problem("g", shape, bcs, (0.02, 0.011), 0.05, "brusselator", BRUSS, 1, seed=n,
                         ic_args={"base": 0.5, "amp": 0.3})
        names, splits = check(prob)
        assert splits[ax] == general_split(n), splits
        assert names[ax].startswith("kr_"), names


@pytest.mark.parametrize("n", GENERAL)
def test_general_line_f32_complex_and_etd1(n):
    """FP32 (1e-5), complex CGL (1e-12) and the first-order scheme (1e-12)
    on general lines, with one species and with two; three steps of ETD-RDP
    within three times the one-step bound."""
    bc = BCS[n % 3]
    p32 = W.Problem("g32", (n, 7), (bc, "neumann"), (0.01, 0.1), 1e-3, "schnakenberg",
                    {"a": 0.1, "b": 0.9, "gamma": 1.0}, 1, seed=1, ic_args={"base": 0.5, "amp": 0.3})
    check(p32, precision="f32", tol=1e-5)
    pz = W.Problem("gz", (6, n), ("periodic", bc), (0.3 + 0.7j,), 1e-3, "cgl_z", {"beta": 1.3}, 1,
                   seed=2, ic="complex_noise", ic_args={"amp": 0.5})
    check(pz, precision="c128")
    pe = W.Problem("ge", (n, 5), (bc, "dirichlet"), (0.2,), 0.02, "enzyme", {}, 1, seed=3,
                   ic_args={"base": 0.5, "amp": 0.3})
    check(pe, scheme="etd1")
    check(pe, nsteps=3, tol=3e-12)


def test_general_lines_many_steps():
    """50 steps of a 2-D problem with general lines on both axes (Gray-Scott
    on 361 x 79, periodic x Neumann): rel-L2 and pointwise <= 1e-10."""
    prob = W.Problem("g50", (361, 79), ("periodic", "neumann"), (2e-5, 1e-5), 1.0, "gray_scott",
                     {"F": 0.04, "kappa": 0.06}, 50, h=(0.01, 0.01), seed=4,
                     ic_args={"base": 0.5, "amp": 0.3})
    check(prob, nsteps=50, tol=1e-10)


def test_general_axes_refuse_reverse_mode_and_single_solves():
    import torch
    from paper_2001_11220_amd import etd
    e = etd.EtdRdp((79, 16), ("dirichlet", "neumann"), (0.02, 0.011), 0.05, "brusselator", BRUSS)
    x = torch.zeros((1, 16, 79), dtype=torch.float64, device="cuda")
    with pytest.raises(etd.EtdError) as ei:
        e.apply_solve(x, axis=1, sigma=0, gamma=3)
    assert ei.value.status == etd.ETD_ERR_UNSUPPORTED
    e.apply_solve(x, axis=2, sigma=0, gamma=3)  # the regular axis still solves
    e.close()


def test_enzyme_p79_grid_against_oracle_and_observed_order():
    """Section 8.1's enzyme grid (unit square, homogeneous Dirichlet,
    h = 0.0125: 79 interior points per axis, D = 0.2, initial value one,
    T = 1) on the GPU: each of the printed step sizes k = 1/20 ... 1/160
    against the oracle (1e-10), and the error against a k = 1/1280 GPU run
    decaying at second order."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    n = 79
    prob = W.Problem("enz", (n, n), ("dirichlet", "dirichlet"), (0.2,), 1.0, "enzyme", {}, 1)
    U0 = np.ones((1, n, n))
    runs = {}
    for nst in (20, 40, 80, 160, 1280):
        p = W.Problem("enz", prob.shape, prob.bcs, prob.D, 1.0 / nst, "enzyme", {}, nst)
        runs[nst], names, _ = run(p, U0, nst)
        assert names[0].startswith("kr_") and names[1].startswith("kr_"), names
        if nst <= 160:
            ref = O.etd_rdp_if_run(U0, 1.0 / nst, [0.2], ["dirichlet"] * 2, list(p.hs()), "enzyme", {}, nst)
            e2, em = rel_l2(runs[nst], ref), rel_max(runs[nst], ref)
            print(f"[enzyme p=79] k=1/{nst} rel_l2={e2:.2e} rel_max={em:.2e}", flush=True)
            assert e2 <= 1e-10 and em <= 1e-10, (nst, e2, em)
    errs = [np.abs(runs[nst] - runs[1280]).max() for nst in (20, 40, 80, 160)]
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    lo = min(gold["enzyme_eoc_etd_rdp_if"]["value"]) - 0.15
    hi = max(gold["enzyme_eoc_etd_rdp_if"]["value"]) + 0.05
    print(f"[enzyme p=79] errors {errs} EOC {eoc}", flush=True)
    assert np.all(eoc > lo) and np.all(eoc < hi), eoc
