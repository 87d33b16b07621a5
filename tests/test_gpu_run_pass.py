"""The per-pass entry points (etd_rdp_run_pass, _f32, _z), which bench.py
times one by one: running passes 1..d in order equals one full step bit for
bit (the same kernels on the same arrays), in every dimension, precision
and scheme."""

import numpy as np
import pytest

from paper_2001_11220_amd import workloads as W

pytestmark = pytest.mark.gpu

GS = {"F": 0.04, "kappa": 0.06}


def _p1(n, bc):
    return W.Problem("t1", (n,), (bc,), (2e-5, 1e-5), 1.0, "gray_scott", GS, 1, seed=0, ic="uniform_noise",
                     ic_args={"base": 0.5, "amp": 0.3})


CASES = [
    (lambda: _p1(200, "periodic"), "f64", "rdp"),
    (lambda: _p1(96, "dirichlet"), "f32", "rdp"),
    (lambda: W.brusselator2d(n=64), "f64", "rdp"),
    (lambda: W.brusselator2d(n=64), "f32", "etd1"),
    (lambda: W.cgl2d_complex(n=40), "c128", "rdp"),
    (lambda: W.grayscott3d(shape=(64, 48, 40)), "f64", "rdp"),
    (lambda: W.grayscott3d(shape=(64, 48, 40)), "f64", "etd1"),
    (lambda: W.grayscott3d(n=64), "f32", "rdp"),
    (lambda: W.cgl3d_complex(n=24), "c128", "rdp"),
    (lambda: W.grayscott3d(shape=(512, 64, 48)), "f64", "rdp"),   # streamed, m = 8
    (lambda: W.grayscott3d(n=256), "f64", "rdp"),                  # the benchmark shape
    (lambda: W.grayscott3d(n=256), "f32", "rdp"),
    (lambda: W.cgl3d_complex(shape=(200, 40, 24)), "c128", "rdp"),  # streamed complex
    (lambda: W.grayscott4d(n=12), "f64", "rdp"),
    (lambda: W.grayscott4d(shape=(16, 12, 10, 8)), "f32", "rdp"),
]


IDS = [
        "1d-200-periodic-f64", "1d-96-dirichlet-f32", "2d-64-f64", "2d-64-f32-etd1", "2d-40-c128",
        "3d-64x48x40-f64", "3d-64x48x40-f64-etd1", "3d-64-f32", "3d-24-c128",
        "3d-512x64x48-streamed-f64", "3d-256-twoline-f64", "3d-256-twoline-f32",
        "3d-200x40x24-streamed-c128", "4d-12-f64", "4d-16x12x10x8-f32"]


@pytest.mark.parametrize("make,prec,scheme", CASES, ids=IDS)
def test_passes_in_order_equal_one_step(make, prec, scheme):
    import torch
    from paper_2001_11220_amd.etd import EtdRdp
    prob = make()
    d = len(prob.shape)
    print(f"[run_pass] {prob.name} {prob.shape} {prec} {scheme}", flush=True)
    e = EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params, h=prob.h, shift=prob.shift,
               scheme=scheme, precision=prec)
    u0 = torch.from_numpy(np.ascontiguousarray(prob.initial())).cuda()
    if prec == "f32":
        u0 = u0.float()
    a = u0.clone()
    e.step(a, 1)
    b = u0.clone()
    for p in range(1, d + 1):
        e.run_pass(b, p)
    torch.cuda.synchronize()
    assert not torch.equal(a, u0)
    assert torch.equal(a, b)
    e.close()
