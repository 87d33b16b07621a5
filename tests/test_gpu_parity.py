"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: rel-L2 <= 1e-12 after one step, <= 1e-10 after 100 steps (FP64),
and the same bound on the largest pointwise error relative to the largest
value (a norm alone would let one cell be off by up to tol * sqrt(N) of it);
single line solves agree to 1e-13 relative (max norm)."""

import math

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


def rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def assert_close(got, ref, tol, label=""):
    """rel-L2 and the largest pointwise error (relative to max |ref|), both
    within tol."""
    e2, em = rel_l2(got, ref), rel_max(got, ref)
    print(f"[parity] {label} rel_l2={e2:.2e} rel_max={em:.2e}", flush=True)
    assert e2 < tol and em < tol, (e2, em, tol)


def make(prob, scheme="rdp", lines_per_wave="auto"):
    return _etd().EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params,
                         h=prob.h, shift=prob.shift, scheme=scheme, lines_per_wave=lines_per_wave)


def gpu_run(prob, u0, nsteps, scheme="rdp", lines_per_wave="auto"):
    torch = _torch()
    e = make(prob, scheme, lines_per_wave)
    u = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
    e.step(u, nsteps)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def oracle_run(prob, u0, nsteps):
    return O.etd_rdp_if_run(u0, prob.k, prob.D, prob.bcs, prob.hs(), prob.model,
                            prob.oracle_params(), nsteps)


def P(shape, bcs, D=(0.02, 0.011), k=0.05, model="brusselator", params=None, shift=None, ic="uniform_noise",
      h=None, seed=0):
    params = params if params is not None else {"a": 1.0, "b": 3.4}
    return W.Problem("t", tuple(shape), tuple(bcs), tuple(D), k, model, params, 1, h=h, shift=shift,
                     seed=seed, ic=ic, ic_args={"base": 0.5, "amp": 0.3})


# ---------------------------------------------------------------------------
# Line solves alone
# ---------------------------------------------------------------------------

SOLVE_SHAPES = [
    (96, 40, 24),     # chunk lengths 2, 1, 1
    (128, 33, 160),   # 2, 1, 4 ; 33 lines per tile row -> ragged tail
    (512, 12, 20),    # 8, ...
    (5, 7, 384),      # tiny contiguous axis, chunk 6 on axis 3
]


@pytest.mark.parametrize("shape", SOLVE_SHAPES)
@pytest.mark.parametrize("bc", ["dirichlet", "neumann", "periodic"])
def test_line_solve_matches_oracle(shape, bc):
    torch = _torch()
    prob = P(shape, (bc,) * 3, D=(0.7, 0.013), k=0.37)  # r from ~0.03 to ~7e4
    e = make(prob)
    rng = np.random.default_rng(11)
    x0 = rng.standard_normal((1,) + tuple(shape[::-1]))
    hs = prob.hs()
    for axis in (1, 2, 3):
        for sigma in (0, 1):
            for gamma in (1, 3, 4):
                x = torch.from_numpy(x0.copy()).cuda()
                e.apply_solve(x, axis, sigma, gamma)
                torch.cuda.synchronize()
                coef = prob.k * prob.D[sigma] / gamma
                ref = O.solve_axis(x0, axis, [coef], bc, hs[axis - 1])
                err = np.abs(x.cpu().numpy() - ref).max() / np.abs(ref).max()
                # Both sides are backward stable; the forward error of either
                # is bounded by a modest multiple of eps * cond(M), and
                # cond(M) <= 1 + 4r with r = coef / h^2.
                r = coef / hs[axis - 1] ** 2
                tol = max(1e-13, 10 * np.finfo(float).eps * (1 + 4 * r))
                assert err < tol, (axis, sigma, gamma, err, tol)


def test_line_solve_stiff_dirichlet_512():
    """r = k D / h^2 ~ 263 (the 512^3 Schnakenberg lines)."""
    torch = _torch()
    prob = P((512, 3, 2), ("dirichlet",) * 3, D=(1.0, 10.0), k=1e-4)
    e = make(prob)
    x0 = np.random.default_rng(3).standard_normal((1, 2, 3, 512))
    for gamma in (1, 3, 4):
        x = torch.from_numpy(x0.copy()).cuda()
        e.apply_solve(x, 1, 1, gamma)
        torch.cuda.synchronize()
        ref = O.solve_axis(x0, 1, [prob.k * 10.0 / gamma], "dirichlet", prob.hs()[0])
        assert np.abs(x.cpu().numpy() - ref).max() / np.abs(ref).max() < 1e-13


# ---------------------------------------------------------------------------
# Passes against the oracle's intermediates
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("bcs", [("neumann", "periodic", "dirichlet"), ("periodic",) * 3])
def test_pass_intermediates_3d(bcs):
    torch = _torch()
    prob = P((64, 40, 24), bcs, model="gray_scott", params={"F": 0.04, "kappa": 0.06}, D=(0.02, 0.01), k=0.5)
    u0 = prob.initial()
    ref = O.step_intermediates(u0, prob.k, prob.D, prob.bcs, prob.hs(), prob.model, prob.oracle_params())
    e = make(prob)
    for npass, keys in ((1, ("cU1", "cf1", "y1")), (2, ("cU2", "cf2", "y2"))):
        u = torch.from_numpy(u0.copy()).cuda()
        e.debug_passes(u, npass)
        torch.cuda.synchronize()
        got = [t.cpu().numpy() for t in e.carried(npass)]
        for g, key in zip(got, keys):
            assert rel_l2(g, ref[key]) < 1e-13, (npass, key, rel_l2(g, ref[key]))


# ---------------------------------------------------------------------------
# Whole steps
# ---------------------------------------------------------------------------

ONE_STEP = [
    P((64, 64), ("neumann", "neumann")),
    P((96, 80), ("periodic", "dirichlet"), model="gray_scott", params={"F": 0.04, "kappa": 0.06}, k=1.0),
    P((33, 47), ("dirichlet", "periodic"), model="cgl", params={"beta": 1.3}, D=(1.0, 1.0), k=0.05,
      h=(0.5, 0.5)),
    P((40, 24, 33), ("neumann", "periodic", "dirichlet"), model="schnakenberg",
      params={"a": 0.1, "b": 0.9, "gamma": 1.0}, D=(1.0, 10.0), k=1e-3, shift=W.SCHNAK_STEADY,
      ic="gaussian_noise"),
    P((128, 20, 48), ("periodic",) * 3, model="gray_scott", params={"F": 0.04, "kappa": 0.06},
      D=(2e-5, 1e-5), k=1.0, ic="cube_patch"),
    P((24, 32, 256), ("dirichlet",) * 3, model="schnakenberg", params={"a": 0.1, "b": 0.9, "gamma": 1.0},
      D=(1.0, 10.0), k=1e-4, shift=W.SCHNAK_STEADY, ic="gaussian_noise"),
    P((30, 20), ("neumann", "dirichlet"), model="enzyme", params={}, D=(0.2,), k=0.05),
    P((16, 12, 10), ("neumann", "neumann", "periodic"), model="linear",
      params={"C": [[-0.3, 0.2], [0.1, -0.5]]}, D=(0.3, 0.1), k=0.1),
    P((2, 3, 1), ("neumann", "periodic", "dirichlet")),  # smallest line lengths
]

# Lines of 32 m rows, m = 2..8, forced to two lines per wavefront: every
# pass, every boundary condition, one and two species, ragged tile tails.
TWO_LINE = [
    P((256, 12, 10), ("neumann", "periodic", "dirichlet")),
    P((10, 192, 13), ("dirichlet", "periodic", "neumann"), model="gray_scott",
      params={"F": 0.04, "kappa": 0.06}, D=(2e-5, 1e-5), k=1.0, ic="cube_patch"),
    P((12, 160, 224), ("periodic", "neumann", "periodic"), model="schnakenberg",
      params={"a": 0.1, "b": 0.9, "gamma": 1.0}, D=(1.0, 10.0), k=1e-4, shift=W.SCHNAK_STEADY,
      ic="gaussian_noise"),
    P((224, 256), ("periodic", "dirichlet"), model="enzyme", params={}, D=(0.2,), k=0.05),
    P((192, 7), ("neumann", "periodic"), model="cgl", params={"beta": 1.3}, D=(1.0, 1.0), k=0.05,
      h=(0.5, 0.5)),
    # chunks of 2-4 rows (lines of 64, 96, 128)
    P((64, 20, 12), ("periodic", "neumann", "dirichlet")),
    P((9, 96, 7), ("dirichlet", "periodic", "neumann"), model="gray_scott", params={"F": 0.04, "kappa": 0.06},
      D=(2e-5, 1e-5), k=1.0, ic="cube_patch"),
    P((6, 10, 128), ("neumann", "dirichlet", "periodic")),
]


@pytest.mark.parametrize("prob", ONE_STEP, ids=lambda p: f"{p.model}-{'x'.join(map(str, p.shape))}")
def test_one_step_matches_oracle(prob):
    u0 = prob.initial()
    got = gpu_run(prob, u0, 1)
    ref = oracle_run(prob, u0, 1)
    assert_close(got, ref, 1e-12, f"one step {prob.model} {prob.shape}")


@pytest.mark.parametrize("prob", TWO_LINE, ids=lambda p: f"{p.model}-{'x'.join(map(str, p.shape))}")
def test_two_lines_per_wave_matches_oracle(prob):
    e = make(prob, lines_per_wave=2)
    names = [e.pass_kernel(p) for p in range(1, len(prob.shape) + 1)]
    e.close()
    # a two-line kernel runs: a streamed form with 2 lines per wavefront, or
    # pass 1's species-paired form (two waves per line pair)
    assert any(("_s<" in nm and nm.split(", ")[3] == "2") or nm.startswith("k_first_pair<")
               for nm in names), names
    u0 = prob.initial()
    got = gpu_run(prob, u0, 2, lines_per_wave=2)
    ref = oracle_run(prob, u0, 2)
    assert_close(got, ref, 1e-12, f"two lines {prob.model} {prob.shape}")
    one = gpu_run(prob, u0, 2, lines_per_wave=1)
    assert_close(got, one, 1e-13, "two lines vs one line")


def test_brusselator2d_100_steps_full_size():
    prob = W.brusselator2d()
    u0 = prob.initial()
    got = gpu_run(prob, u0, 100)
    ref = oracle_run(prob, u0, 100)
    assert_close(got, ref, 1e-10, "brusselator2d 100 steps")


def test_grayscott3d_100_steps_small():
    prob = W.grayscott3d(n=32, nsteps=100)
    u0 = prob.initial()
    got = gpu_run(prob, u0, 100)
    ref = oracle_run(prob, u0, 100)
    assert_close(got, ref, 1e-10, "grayscott3d 32^3 100 steps")


@pytest.mark.parametrize("shape,lpw", [((48, 40, 20), "auto"), ((160, 12, 224), 2)])
def test_etd1_predictor_matches_oracle(shape, lpw):
    prob = P(shape, ("neumann", "periodic", "dirichlet"))
    u0 = prob.initial()
    got = gpu_run(prob, u0, 1, scheme="etd1", lines_per_wave=lpw)
    ref = O.etd1_if_step(u0, prob.k, prob.D, prob.bcs, prob.hs(), prob.model, prob.oracle_params())
    assert_close(got, ref, 1e-12, f"etd1 {shape}")


def test_determinism_and_step_splitting():
    torch = _torch()
    prob = P((64, 48, 40), ("periodic", "neumann", "dirichlet"), model="gray_scott",
             params={"F": 0.04, "kappa": 0.06}, k=0.5)
    e = make(prob)
    u0 = torch.from_numpy(prob.initial()).cuda()
    a = u0.clone()
    e.step(a, 5)
    b = u0.clone()
    e.step(b, 3)
    e.step(b, 2)
    c = u0.clone()
    e.step(c, 0)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(c, u0)


def test_fixed_point_and_zero_diffusion():
    prob = P((40, 24, 16), ("neumann",) * 3, D=(0.0, 0.0), k=0.07)
    u0 = prob.initial()
    got = gpu_run(prob, u0, 1)
    F = lambda X: O.reaction("brusselator", prob.params, X)
    heun = u0 + 0.5 * prob.k * (F(u0) + F(u0 + prob.k * F(u0)))
    assert rel_l2(got, heun) < 1e-13
    ss = np.stack([np.full((16, 24, 40), 1.0), np.full((16, 24, 40), 3.4)])
    prob2 = P((40, 24, 16), ("neumann",) * 3)
    assert np.abs(gpu_run(prob2, ss, 3) - ss).max() < 1e-13


# ---------------------------------------------------------------------------
# Full-size workloads in the benchmark's launch configuration (sampled)
# ---------------------------------------------------------------------------

def _sampled_step_reference(prob, u0, x0s):
    """Oracle step restricted to the planes x = x0 (axis 1 index): pass 1 is
    computed on the whole grid, the remaining axes only on those planes,
    which they do not couple."""
    k, D, bcs, hs = prob.k, prob.D, prob.bcs, prob.hs()
    p = prob.oracle_params()
    f = O.reaction(prob.model, p, u0)
    cU = O.apply_R(u0, 1, k, D, bcs[0], hs[0])[..., x0s]
    cf = O.apply_R(f, 1, k, D, bcs[0], hs[0])[..., x0s]
    y = O.solve_axis(u0 + k * f, 1, k * np.asarray(D), bcs[0], hs[0])[..., x0s]
    d = u0.ndim - 1
    for i in range(2, d + 1):
        y = O.solve_axis(y, i, k * np.asarray(D), bcs[i - 1], hs[i - 1])
    for i in range(2, d):
        cU = O.apply_R(cU, i, k, D, bcs[i - 1], hs[i - 1])
        cf = O.apply_R(cf, i, k, D, bcs[i - 1], hs[i - 1])
    fs = O.reaction(prob.model, p, y)
    f1 = 9 * cU + 2 * k * cf + k * fs
    f2 = 8 * cU + 1.5 * k * cf + 0.5 * k * fs
    return (O.solve_axis(f1, d, k * np.asarray(D) / 3, bcs[d - 1], hs[d - 1])
            - O.solve_axis(f2, d, k * np.asarray(D) / 4, bcs[d - 1], hs[d - 1]))


def test_grayscott3d_full_size_one_step_sampled():
    prob = W.grayscott3d()
    u0 = prob.initial()
    got = gpu_run(prob, u0, 1)
    x0s = [0, 101, 128, 255]
    ref = _sampled_step_reference(prob, u0, x0s)
    assert_close(got[..., x0s], ref, 1e-12, "grayscott3d 256^3 sampled")


def test_schnakenberg3d_full_size_one_step_sampled():
    """512^3 Dirichlet (chunk length 8, r up to ~263), benchmark launch
    configuration; planes x = x0 checked against the oracle."""
    prob = W.schnakenberg3d()
    u0 = prob.initial()
    got = gpu_run(prob, u0, 1)
    x0s = [0, 255, 511]
    ref = _sampled_step_reference(prob, u0, x0s)
    assert_close(got[..., x0s], ref, 1e-12, "schnakenberg3d 512^3 sampled")


def test_grayscott4d_full_size_one_step_sampled():
    """64^4 periodic (two lines of 32 two-row chunks per wavefront on every
    axis), benchmark launch configuration; planes x = x0 checked against the
    oracle."""
    prob = W.grayscott4d()
    u0 = prob.initial()
    got = gpu_run(prob, u0, 1)
    x0s = [0, 31, 63]
    ref = _sampled_step_reference(prob, u0, x0s)
    assert_close(got[..., x0s], ref, 1e-12, "grayscott4d 64^4 sampled")


def test_grayscott5d_full_size_one_step_sampled():
    """32^5 periodic (four lines of 16 two-row chunks per wavefront on every
    axis, cyclic layouts), benchmark launch configuration; planes x = x0
    checked against the oracle."""
    prob = W.grayscott5d()
    u0 = prob.initial()
    got = gpu_run(prob, u0, 1)
    x0s = [0, 15, 31]
    ref = _sampled_step_reference(prob, u0, x0s)
    assert_close(got[..., x0s], ref, 1e-12, "grayscott5d 32^5 sampled")


def test_f32_full_size_one_step_sampled_against_oracle():
    """The 256^3 workload in FP32 (two lines per wavefront, non-temporal
    stores), one step on the planes x = x0 against the FP64 oracle: the
    single-precision tolerance, 1e-5, in rel-L2 and in the largest pointwise
    error."""
    torch = _torch()
    prob = W.grayscott3d()
    u0 = prob.initial()
    e = _etd().EtdRdp(prob.shape, prob.bcs, prob.D, prob.k, prob.model, prob.params, precision="f32")
    u = torch.from_numpy(u0).cuda().float()
    e.step(u, 1)
    torch.cuda.synchronize()
    x0s = [0, 128, 255]
    got = u[..., x0s].cpu().numpy().astype(np.float64)
    e.close()
    ref = _sampled_step_reference(prob, u0, x0s)
    assert_close(got, ref, 1e-5, "grayscott3d 256^3 FP32 sampled")
