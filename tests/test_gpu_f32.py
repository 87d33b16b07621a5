"""GPU parity of the single-precision forward path (etd_rdp_step_f32)
against the FP64 oracle.

Tolerance: one step agrees with the oracle to rel-L2 <= 1e-5 (measured
1.0e-6 to 2.9e-6 over every case here, up to r = k D / h^2 of ~6e4).  For
information the tests print the condition-number bound
5 eps32 (1 + 4 r_max), eps32 = 2^-24 (both sides are backward-stable line
solves and a solve's forward error is at most its condition number, at most
1 + 4r, times that); it is not what they assert.  Longer runs are checked
against n times the one-step tolerance."""

import numpy as np
import pytest

import oracle as O
from paper_2001_11220_amd import workloads as W

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24


def _torch():
    import torch
    return torch


def _etd():
    from paper_2001_11220_amd import etd
    return etd


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def P(shape, bcs, D=(0.02, 0.011), k=0.05, model="brusselator", params=None, shift=None, ic="uniform_noise",
      h=None):
    params = params if params is not None else {"a": 1.0, "b": 3.4}
    return W.Problem("t", tuple(shape), tuple(bcs), tuple(D), k, model, params, 1, h=h, shift=shift,
                     seed=0, ic=ic, ic_args={"base": 0.5, "amp": 0.3})


def r_max(prob):
    return max(prob.k * d / (h * h) for d in prob.D for h in prob.hs())


def run_f32(prob, u0, nsteps, lines_per_wave="auto"):
    torch = _torch()
    e = _etd().EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params, h=prob.h,
                      shift=prob.shift, precision="f32", lines_per_wave=lines_per_wave)
    u = torch.from_numpy(np.ascontiguousarray(u0, dtype=np.float32)).cuda()
    e.step(u, nsteps)
    torch.cuda.synchronize()
    names = [e.pass_kernel(p) for p in range(1, len(prob.shape) + 1)]
    e.close()
    assert all(nm.endswith(", float>") for nm in names), names
    return u.cpu().numpy().astype(np.float64)


CASES = [
    (P((64, 64), ("neumann", "neumann")), "auto"),
    (P((96, 80), ("periodic", "dirichlet"), model="gray_scott", params={"F": 0.04, "kappa": 0.06}, k=1.0), "auto"),
    (P((40, 24, 33), ("neumann", "periodic", "dirichlet"), model="schnakenberg",
       params={"a": 0.1, "b": 0.9, "gamma": 1.0}, D=(1.0, 10.0), k=1e-3, shift=W.SCHNAK_STEADY,
       ic="gaussian_noise"), "auto"),
    (P((128, 20, 48), ("periodic",) * 3, model="gray_scott", params={"F": 0.04, "kappa": 0.06},
       D=(2e-5, 1e-5), k=1.0, ic="cube_patch"), "auto"),
    (P((30, 20), ("neumann", "dirichlet"), model="enzyme", params={}, D=(0.2,), k=0.05), "auto"),
    (P((16, 12, 10), ("neumann", "neumann", "periodic"), model="linear",
       params={"C": [[-0.3, 0.2], [0.1, -0.5]]}, D=(0.3, 0.1), k=0.1), "auto"),
    (P((2, 3, 1), ("neumann", "periodic", "dirichlet")), "auto"),             # smallest line lengths
    (P((24, 32, 256), ("dirichlet",) * 3, model="schnakenberg", params={"a": 0.1, "b": 0.9, "gamma": 1.0},
       D=(1.0, 10.0), k=1e-4, shift=W.SCHNAK_STEADY, ic="gaussian_noise"), "auto"),
    (P((33, 47), ("dirichlet", "periodic"), model="cgl", params={"beta": 1.3}, D=(1.0, 1.0), k=0.05,
       h=(0.5, 0.5)), "auto"),
    (P((512, 12, 10), ("dirichlet", "neumann", "periodic")), "auto"),          # chunk length 8, streamed
    (P((256, 12, 10), ("neumann", "periodic", "dirichlet")), 2),              # two lines per wavefront
    (P((12, 160, 224), ("periodic", "neumann", "periodic"), model="schnakenberg",
       params={"a": 0.1, "b": 0.9, "gamma": 1.0}, D=(1.0, 10.0), k=1e-4, shift=W.SCHNAK_STEADY,
       ic="gaussian_noise"), 2),
]


@pytest.mark.parametrize("prob,lpw", CASES, ids=lambda c: f"{c.model}-{'x'.join(map(str, c.shape))}"
                         if hasattr(c, "model") else str(c))
def test_one_step_f32_matches_oracle(prob, lpw):
    u0 = prob.initial()
    got = run_f32(prob, u0, 1, lpw)
    ref = O.etd_rdp_if_run(u0, prob.k, prob.D, prob.bcs, prob.hs(), prob.model, prob.oracle_params(), 1)
    tol = 1e-5
    err = rel_l2(got, ref)
    print(f"[f32 one step] {prob.model} {prob.shape} rel_l2={err:.2e} tol={tol:.2e} "
          f"(condition bound {5 * EPS32 * (1 + 4 * r_max(prob)):.1e})", flush=True)
    assert err <= tol, (err, tol)


def test_f32_100_steps_error_curve():
    prob = W.grayscott3d(n=32, nsteps=100)
    u0 = prob.initial()
    torch = _torch()
    e = _etd().EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params, h=prob.h,
                      shift=prob.shift, precision="f32")
    u = torch.from_numpy(u0.astype(np.float32)).cuda()
    ref = u0.copy()
    errs = []
    for chunk in (10,) * 10:
        e.step(u, chunk)
        ref = O.etd_rdp_if_run(ref, prob.k, prob.D, prob.bcs, prob.hs(), prob.model,
                               prob.oracle_params(), chunk)
        torch.cuda.synchronize()
        errs.append(rel_l2(u.cpu().numpy().astype(np.float64), ref))
    e.close()
    print("[f32 error curve] every 10 steps:", " ".join(f"{v:.1e}" for v in errs), flush=True)
    # rounding errors accumulate at most linearly in the step count: n steps
    # within n times the one-step tolerance (measured 5.9e-6 after 100)
    assert all(e <= 10 * (i + 1) * 1e-5 for i, e in enumerate(errs)), errs


def test_f32_matches_f64_gpu_at_full_size():
    torch = _torch()
    prob = W.grayscott3d()  # 256^3, two lines per wavefront, non-temporal stores
    u0 = prob.initial()
    e64 = _etd().EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params, h=prob.h,
                        shift=prob.shift)
    e32 = _etd().EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params, h=prob.h,
                        shift=prob.shift, precision="f32")
    assert e32.pass_kernel(2) == "k_mid_s<8, 2, 32, 2, true, float>"
    u64 = torch.from_numpy(u0).cuda()
    u32 = u64.float()
    e64.step(u64, 1)
    e32.step(u32, 1)
    torch.cuda.synchronize()
    err = float(torch.linalg.norm(u32.double() - u64) / torch.linalg.norm(u64))
    e64.close()
    e32.close()
    print(f"[f32 vs f64 GPU, 256^3] rel_l2={err:.2e}", flush=True)
    assert err <= 1e-5, err


def test_precision_mismatch_is_refused():
    torch = _torch()
    etd = _etd()
    prob = P((64, 64), ("neumann", "neumann"))
    e32 = etd.EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params, precision="f32")
    u64 = torch.zeros((2, 64, 64), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        e32.step(u64, 1)  # the binding checks the dtype first
    u32 = torch.zeros((2, 64, 64), dtype=torch.float32, device="cuda")
    import ctypes
    rc = etd.lib.etd_rdp_step(e32._ctx, ctypes.c_void_p(u32.data_ptr()), ctypes.c_void_p(e32._ws_ptr()),
                              e32.ws_bytes, 1, None)
    assert rc == etd.ETD_ERR_ARG
    with pytest.raises(etd.EtdError):
        e32.adjoint(u64, u64)
    e32.close()


def test_f32_matches_f64_gpu_at_512():
    """The 512^3 Dirichlet workload (one line per wavefront, streamed
    16-line tiles), one step in FP32 against the FP64 GPU step.  Both
    states are stored as the shifted unknown w = u - u* of size 1e-3, so the
    error is measured relative to w."""
    torch = _torch()
    prob = W.schnakenberg3d()
    u0 = prob.initial()
    mk = lambda prec: _etd().EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params,
                                    h=prob.h, shift=prob.shift, precision=prec)
    e64, e32 = mk("f64"), mk("f32")
    assert e32.pass_kernel(2) == "k_mid_s<8, 2, 16, 1, true, float>"
    u64 = torch.from_numpy(u0).cuda()
    u32 = u64.float()
    e64.step(u64, 1)
    e32.step(u32, 1)
    torch.cuda.synchronize()
    err = float(torch.linalg.norm(u32.double() - u64) / torch.linalg.norm(u64))
    e64.close()
    e32.close()
    r = max(prob.k * d / h ** 2 for d in prob.D for h in prob.hs())
    tol = 1e-5
    print(f"[f32 vs f64 GPU, 512^3] rel_l2={err:.2e} tol={tol:.2e} "
          f"(condition bound {5 * EPS32 * (1 + 4 * r):.1e})", flush=True)
    assert err <= tol, (err, tol)
