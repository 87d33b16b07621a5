"""Eight lines per wavefront (ETD_LINES_EIGHT): lines of n = 8 m rows
(2 <= m <= 8, n <= 64) solved as 8 chunks of m rows, eight lines per
wavefront (three reduction levels per solve), on every kind of pass,
against the FP64 oracle (rel-L2 and largest pointwise error <= 1e-12 per
step; FP32 1e-5) and against the one-line chunking (rounding only: 1e-13, or
4 eps kappa, kappa = 1 + 4 max k D / h^2)."""

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
    # (shape, bcs, D, k, model, params); lengths 16 .. 64 = 8 m
    ((64, 48, 32), ("neumann", "periodic", "dirichlet"), (0.02, 0.011), 0.05, "brusselator", BRUSS),
    ((40, 56, 24), ("dirichlet", "neumann", "periodic"), (0.02, 0.011), 0.05, "brusselator", BRUSS),
    ((16, 64), ("periodic", "neumann"), (2e-5, 1e-5), 1.0, "gray_scott", {"F": 0.04, "kappa": 0.06}),
    ((32, 48, 64, 16), ("periodic", "dirichlet", "neumann", "periodic"), (0.3,), 0.04, "linear",
     {"C": [[-0.7]]}),
    ((32, 24, 16, 40, 8), ("neumann", "periodic", "dirichlet", "periodic", "neumann"), (0.02, 0.011), 0.05,
     "brusselator", BRUSS),
    ((64,), ("neumann",), (0.2,), 0.02, "enzyme", {}),
    ((64, 40, 96), ("dirichlet", "dirichlet", "neumann"), (1.0, 10.0), 1e-3, "schnakenberg",
     {"a": 0.1, "b": 0.9, "gamma": 1.0}),
]


def _eight(n):
    return n % 8 == 0 and 2 <= n // 8 <= 8


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[0])))
def test_eight_lines_per_wave_matches_oracle(case):
    shape, bcs, D, k, model, params = case
    prob = W.Problem("f8", shape, bcs, D, k, model, params, 1, seed=len(shape),
                     ic_args={"base": 0.5, "amp": 0.3})
    u0 = prob.initial()
    got, names, splits = run(prob, u0, 2, 8)
    for a, n in enumerate(shape):
        if _eight(n):
            assert splits[a] == (n // 8, 8), (a, splits)
            # streamed 128-line tiles, or pass 1's species-paired form
            assert (", 128, 8, " in names[a] or
                    (names[a].startswith("k_first_pair<") and names[a].split(", ")[2] == "8")), (a, names)
    ref = O.etd_rdp_if_run(u0, k, D, bcs, prob.hs(), model, prob.oracle_params(), 2)
    e2, em = rel_l2(got, ref), rel_max(got, ref)
    print(f"[eight lines] {shape} {bcs} {model} {names} rel_l2={e2:.2e} rel_max={em:.2e}", flush=True)
    assert e2 <= 2e-12 and em <= 2e-12, (e2, em)
    one, _, _ = run(prob, u0, 2, 1)
    kappa = 1.0 + 4.0 * max(k * d / h ** 2 for d in D for h in prob.hs())
    assert rel_max(got, one) <= max(1e-13, 4.0 * np.finfo(np.float64).eps * kappa), kappa


@pytest.mark.parametrize("prec,scheme", [("f32", "rdp"), ("f64", "etd1")])
def test_eight_lines_f32_and_etd1(prec, scheme):
    shape, bcs, D, k, model, params = CASES[1]
    prob = W.Problem("f8", shape, bcs, D, k, model, params, 1, seed=7, ic_args={"base": 0.5, "amp": 0.3})
    u0 = prob.initial()
    got, names, _ = run(prob, u0, 1, 8, precision=prec, scheme=scheme)
    step = O.etd1_if_step if scheme == "etd1" else O.etd_rdp_if_step
    ref = step(u0, k, D, bcs, prob.hs(), model, prob.oracle_params())
    tol = 1e-5 if prec == "f32" else 1e-12
    e2, em = rel_l2(got, ref), rel_max(got, ref)
    print(f"[eight lines {prec} {scheme}] {names} rel_l2={e2:.2e} rel_max={em:.2e}", flush=True)
    assert e2 <= tol and em <= tol, (e2, em)


def test_eight_lines_reverse_step_matches_oracle():
    """A forward pass at eight lines per wavefront: the reverse step's
    recompute runs it, its reverse passes run the two-line (or one-line)
    chunking on their own table set."""
    import torch
    from paper_2001_11220_amd import etd
    shape, bcs = (64, 48, 32), ("neumann", "periodic", "dirichlet")
    D, k = (0.02, 0.011), 0.05
    e = etd.EtdRdp(shape, bcs, D, k, "brusselator", BRUSS, lines_per_wave=8)
    rng = np.random.default_rng(4)
    U = np.stack([1.0 + 0.2 * rng.random(shape[::-1]), 3.4 + 0.2 * rng.random(shape[::-1])])
    lam = rng.standard_normal(U.shape)
    lo, g = e.adjoint(torch.from_numpy(U).cuda(), torch.from_numpy(lam).cuda())
    torch.cuda.synchronize()
    hs = W.Problem("t", shape, bcs, (1.0,), 1.0, "linear", {}, 1).hs()
    lo_o, gD, gth = O.adjoint_step(U, lam, k, D, bcs, hs, "brusselator", BRUSS)
    assert rel_l2(lo.cpu().numpy(), lo_o) <= 1e-11
    go = np.concatenate([gD, gth])
    assert np.all(np.abs(g.cpu().numpy() - go) <= 1e-9 * np.abs(go) + 1e-12 * np.abs(go).max()), (g, go)
    e.close()
