"""Four lines per wavefront (ETD_LINES_FOUR): lines of n = 16 m rows
(2 <= m <= 8) solved as 16 chunks of m rows, four lines per wavefront, on
every kind of pass, against the FP64 oracle (rel-L2 and largest pointwise
error <= 1e-12 per step; FP32 1e-5) and against the one-line chunking
(rounding only: 1e-13, or 4 eps kappa for stiff lines, kappa the line
matrix's condition number bound 1 + 4 max k D / h^2)."""

import numpy as np
import pytest

import oracle as O
from paper_2001_11220_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def run(prob, u0, nsteps, lpw, precision="f64", scheme="rdp"):
    import torch
    from paper_2001_11220_amd import etd
    e = etd.EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params, h=prob.h,
                   lines_per_wave=lpw, precision=precision, scheme=scheme)
    names = [e.pass_kernel(p) for p in range(1, len(prob.shape) + 1)]
    splits = [e.line_split(a) for a in range(1, len(prob.shape) + 1)]
    u = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
    if precision == "f32":
        u = u.float()
    e.step(u, nsteps)
    torch.cuda.synchronize()
    e.close()
    return u.cpu().numpy().astype(np.float64), names, splits


BRUSS = {"a": 1.0, "b": 3.4}
CASES = [
    # (shape, bcs, D, k, model, params)
    ((64, 48, 32), ("neumann", "periodic", "dirichlet"), (0.02, 0.011), 0.05, "brusselator", BRUSS),
    ((128, 96, 80), ("dirichlet", "neumann", "periodic"), (0.02, 0.011), 0.05, "brusselator", BRUSS),
    ((112, 64), ("periodic", "neumann"), (2e-5, 1e-5), 1.0, "gray_scott", {"F": 0.04, "kappa": 0.06}),
    ((32, 48, 64, 16), ("periodic", "dirichlet", "neumann", "periodic"), (0.3,), 0.04, "linear",
     {"C": [[-0.7]]}),
    ((96,), ("neumann",), (0.2,), 0.02, "enzyme", {}),
    ((64, 40, 128), ("dirichlet", "dirichlet", "neumann"), (1.0, 10.0), 1e-3, "schnakenberg",
     {"a": 0.1, "b": 0.9, "gamma": 1.0}),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[0])))
def test_four_lines_per_wave_matches_oracle(case):
    shape, bcs, D, k, model, params = case
    prob = W.Problem("f4", shape, bcs, D, k, model, params, 1, seed=len(shape),
                     ic_args={"base": 0.5, "amp": 0.3})
    u0 = prob.initial()
    got, names, splits = run(prob, u0, 2, 4)
    for a, n in enumerate(shape):
        if n % 16 == 0 and 2 <= n // 16 <= 8:
            assert splits[a] == (n // 16, 16), (a, splits)
            # streamed 64-line tiles, or pass 1's species-paired form
            assert (", 64, 4, " in names[a] or
                    (names[a].startswith("k_first_pair<") and names[a].split(", ")[2] == "4")), (a, names)
    ref = O.etd_rdp_if_run(u0, k, D, bcs, prob.hs(), model, prob.oracle_params(), 2)
    e2, em = rel_l2(got, ref), rel_max(got, ref)
    print(f"[four lines] {shape} {bcs} {model} {names} rel_l2={e2:.2e} rel_max={em:.2e}", flush=True)
    assert e2 <= 2e-12 and em <= 2e-12, (e2, em)
    # the chunkings differ only in rounding: each solve's forward error is at
    # most the line matrix's condition number kappa times eps
    one, _, _ = run(prob, u0, 2, 1)
    kappa = 1.0 + 4.0 * max(k * d / h ** 2 for d in D for h in prob.hs())
    assert rel_max(got, one) <= max(1e-13, 4.0 * np.finfo(np.float64).eps * kappa), kappa


@pytest.mark.parametrize("prec,scheme", [("f32", "rdp"), ("f64", "etd1")])
def test_four_lines_f32_and_etd1(prec, scheme):
    shape, bcs, D, k, model, params = CASES[1]
    prob = W.Problem("f4", shape, bcs, D, k, model, params, 1, seed=7, ic_args={"base": 0.5, "amp": 0.3})
    u0 = prob.initial()
    got, names, _ = run(prob, u0, 1, 4, precision=prec, scheme=scheme)
    step = O.etd1_if_step if scheme == "etd1" else O.etd_rdp_if_step
    ref = step(u0, k, D, bcs, prob.hs(), model, prob.oracle_params())
    tol = 1e-5 if prec == "f32" else 1e-12
    e2, em = rel_l2(got, ref), rel_max(got, ref)
    print(f"[four lines {prec} {scheme}] {names} rel_l2={e2:.2e} rel_max={em:.2e}", flush=True)
    assert e2 <= tol and em <= tol, (e2, em)
