"""Seeded synthetic workloads (problem definitions and initial data).

This module holds no arithmetic of the scheme: it only states the problems
(grid, boundary conditions, coefficients, reaction parameters, step count)
and draws their initial data from ``numpy.random.default_rng(seed)``.  The
same arrays feed the GPU library and the CPU oracle.

Workloads (the paper uses no external dataset; these stand in for the
benchmark configurations of the build):

* ``brusselator2d``   2-D Brusselator a=1, b=3.4, D=(0.02, 0.02), n=64^2,
  Neumann (h = 1/63), k = 0.01, 100 steps, u, v = 0.5 + 0.1 U[0,1).
* ``grayscott3d``     3-D Gray-Scott F=0.04, kappa=0.06, D=(2e-5, 1e-5),
  n=256^3 periodic (h = 1/256), k = 1, 500 steps; u = 1, v = 0 except a
  centred cube of side n/8 with u = 1 - 0.25 xi, v = 0.25 xi'.
* ``schnakenberg3d``  3-D Schnakenberg a=0.1, b=0.9, gamma=1, D=(1, 10),
  n=512^3, homogeneous Dirichlet on w = u - u* with u* = (a+b, b/(a+b)^2)
  (h = 1/513), k = 1e-4, 200 steps, w = 1e-3 N(0,1).
* ``schnakenberg3d_adjoint``  128^3 Neumann (h = 1/127), k = 1e-3, 400 steps,
  u = u* + 1e-3 N(0,1) (unshifted); the loss's target is the same run with
  (Du, Dv, a, b) perturbed by up to 5 % (``gradient_target``).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Optional, Sequence, Tuple

import numpy as np


@dataclass
class Problem:
    name: str
    shape: Tuple[int, ...]          # (n_1, ..., n_d)
    bcs: Tuple[str, ...]            # per axis
    D: Tuple[float, ...]
    k: float
    model: str
    params: Dict[str, float]
    nsteps: int
    h: Optional[Tuple[float, ...]] = None   # None: unit-domain default
    shift: Optional[Tuple[float, ...]] = None
    seed: int = 0
    ic: str = "uniform_noise"
    ic_args: Dict[str, float] = field(default_factory=dict)

    @property
    def s(self) -> int:
        return len(self.D)

    @property
    def cells(self) -> int:
        return int(np.prod(self.shape))

    @property
    def is_complex(self) -> bool:
        """One complex species (complex diffusion coefficient)."""
        return any(isinstance(v, complex) for v in self.D)

    @property
    def precision(self) -> str:
        return "c128" if self.is_complex else "f64"

    def state_shape(self) -> Tuple[int, ...]:
        return (self.s,) + tuple(self.shape[::-1])

    def hs(self) -> Tuple[float, ...]:
        out = []
        for i, (n, b) in enumerate(zip(self.shape, self.bcs)):
            if self.h is not None and self.h[i]:
                out.append(float(self.h[i]))
            elif b == "dirichlet":
                out.append(1.0 / (n + 1))
            elif b == "neumann":
                out.append(1.0 / (n - 1))
            else:
                out.append(1.0 / n)
        return tuple(out)

    def oracle_params(self) -> Dict[str, float]:
        p = dict(self.params)
        if self.shift is not None:
            p["shift"] = list(self.shift)
        return p

    def initial(self) -> np.ndarray:
        return initial_data(self)


def initial_data(p: Problem) -> np.ndarray:
    """Seeded initial state of shape ``(s, n_d, ..., n_1)`` (float64)."""
    rng = np.random.default_rng(p.seed)
    shp = p.state_shape()
    if p.ic == "uniform_noise":
        base = p.ic_args.get("base", 0.5)
        amp = p.ic_args.get("amp", 0.1)
        return np.stack([base + amp * rng.random(shp[1:]) for _ in range(p.s)])
    if p.ic == "gaussian_noise":
        amp = p.ic_args.get("amp", 1e-3)
        out = amp * rng.standard_normal(shp)
        if "offset" in p.ic_args:
            off = p.ic_args["offset"]
            for i in range(p.s):
                out[i] += off[i]
        return out
    if p.ic == "cube_patch":
        amp = p.ic_args.get("amp", 0.25)
        u = np.ones(shp[1:])
        v = np.zeros(shp[1:])
        sl = []
        for n in shp[1:]:
            side = max(1, n // 8)
            lo = (n - side) // 2
            sl.append(slice(lo, lo + side))
        sl = tuple(sl)
        pshape = u[sl].shape
        u[sl] = 1.0 - amp * rng.random(pshape)
        v[sl] = amp * rng.random(pshape)
        return np.stack([u, v])
    if p.ic == "gaussian_pulses":
        # Section 8.3: exp(-|x - c1|^2 / w) - exp(-|x - c2|^2 / w) on the grid
        # x_i = i h (complex state, zero imaginary part).
        w = p.ic_args.get("width", 1000.0)
        c1, c2 = p.ic_args.get("c1", 50.0), p.ic_args.get("c2", 100.0)
        axes = [np.arange(n) * h for n, h in zip(p.shape, p.hs())]
        grids = np.meshgrid(*axes[::-1], indexing="ij")  # (n_d, ..., n_1)
        r1 = sum((g - c1) ** 2 for g in grids)
        r2 = sum((g - c2) ** 2 for g in grids)
        u = np.exp(-r1 / w) - np.exp(-r2 / w)
        return u[None].astype(np.complex128)
    if p.ic == "gaussian_pulses_2d":
        # Section 8.3, 2-D: exp(-|x - (50, 50)|^2 / w) - exp(-|x - (100, 100)|^2 / w)
        # + exp(-|x - (100, 50)|^2 / w) on the grid x_i = i h.
        w = p.ic_args.get("width", 1000.0)
        x = np.arange(p.shape[0]) * p.hs()[0]
        y = np.arange(p.shape[1]) * p.hs()[1]
        Y, X = np.meshgrid(y, x, indexing="ij")  # (n_2, n_1)
        g = lambda cx, cy: np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / w)
        u = g(50.0, 50.0) - g(100.0, 100.0) + g(100.0, 50.0)
        return u[None].astype(np.complex128)
    if p.ic == "complex_noise":
        # Section 8.3's normal random field: real and imaginary parts
        # standard normal, scaled by amp.
        amp = p.ic_args.get("amp", 1.0)
        return amp * (rng.standard_normal(shp) + 1j * rng.standard_normal(shp))
    raise ValueError(p.ic)


def brusselator2d(n: int = 64, nsteps: int = 100, seed: int = 0) -> Problem:
    return Problem("brusselator2d", (n, n), ("neumann", "neumann"), (0.02, 0.02), 0.01,
                   "brusselator", {"a": 1.0, "b": 3.4}, nsteps, seed=seed,
                   ic="uniform_noise", ic_args={"base": 0.5, "amp": 0.1})


def grayscott3d(n: int = 256, nsteps: int = 500, seed: int = 0, shape=None) -> Problem:
    shape = tuple(shape) if shape is not None else (n, n, n)
    return Problem("grayscott3d", shape, ("periodic",) * 3, (2e-5, 1e-5), 1.0,
                   "gray_scott", {"F": 0.04, "kappa": 0.06}, nsteps, seed=seed,
                   ic="cube_patch", ic_args={"amp": 0.25})


def grayscott4d(n: int = 64, nsteps: int = 100, seed: int = 0, shape=None) -> Problem:
    """The Gray-Scott benchmark system on the periodic unit 4-cube (the
    general-d frame of Section 6), 64^4 cells, same coefficients, k and
    initial-data recipe as the 3-D workload."""
    shape = tuple(shape) if shape is not None else (n, n, n, n)
    return Problem("grayscott4d", shape, ("periodic",) * 4, (2e-5, 1e-5), 1.0,
                   "gray_scott", {"F": 0.04, "kappa": 0.06}, nsteps, seed=seed,
                   ic="cube_patch", ic_args={"amp": 0.25})


def grayscott5d(n: int = 32, nsteps: int = 100, seed: int = 0, shape=None) -> Problem:
    """The same system on the periodic unit 5-cube, 32^5 cells (as many
    cells as the 256^3 workload): the general-d frame with five split
    factors."""
    shape = tuple(shape) if shape is not None else (n,) * 5
    return Problem("grayscott5d", shape, ("periodic",) * 5, (2e-5, 1e-5), 1.0,
                   "gray_scott", {"F": 0.04, "kappa": 0.06}, nsteps, seed=seed,
                   ic="cube_patch", ic_args={"amp": 0.25})


SCHNAK = {"a": 0.1, "b": 0.9, "gamma": 1.0}
SCHNAK_STEADY = (SCHNAK["a"] + SCHNAK["b"], SCHNAK["b"] / (SCHNAK["a"] + SCHNAK["b"]) ** 2)


def schnakenberg3d(n: int = 512, nsteps: int = 200, seed: int = 0, shape=None) -> Problem:
    shape = tuple(shape) if shape is not None else (n, n, n)
    return Problem("schnakenberg3d", shape, ("dirichlet",) * 3, (1.0, 10.0), 1e-4,
                   "schnakenberg", dict(SCHNAK), nsteps, shift=SCHNAK_STEADY, seed=seed,
                   ic="gaussian_noise", ic_args={"amp": 1e-3})


def schnakenberg3d_adjoint(n: int = 128, nsteps: int = 400, seed: int = 0) -> Problem:
    return Problem("schnakenberg3d_adjoint", (n, n, n), ("neumann",) * 3, (1.0, 10.0), 1e-3,
                   "schnakenberg", dict(SCHNAK), nsteps, seed=seed, ic="gaussian_noise",
                   ic_args={"amp": 1e-3, "offset": SCHNAK_STEADY})


def gradient_target(prob: Problem):
    """Parameters of the target run of the gradient workload: theta =
    (Du, Dv, a, b) each multiplied by 1 + 0.05 U[-1, 1), drawn in that order
    from default_rng(seed + 1); gamma is kept.  Returns (D_t, params_t)."""
    rng = np.random.default_rng(prob.seed + 1)
    f = [1.0 + 0.05 * rng.uniform(-1.0, 1.0) for _ in range(4)]
    D_t = (prob.D[0] * f[0], prob.D[1] * f[1])
    params_t = dict(prob.params)
    params_t["a"] = prob.params["a"] * f[2]
    params_t["b"] = prob.params["b"] * f[3]
    return D_t, params_t


CGL_ALPHA, CGL_BETA = 0.5, 1.3


def cgl3d_complex(n: int = 200, nsteps: int = 100, seed: int = 0, shape=None) -> Problem:
    """Complex Ginzburg-Landau on the periodic cube [0, 200]^3 (Section 8.3:
    p = 200, h = 1, k = 1/20, beta = 1.3, Gaussian pulses), with linear
    dispersion alpha = 0.5 (D = 1 + 0.5 i)."""
    shape = tuple(shape) if shape is not None else (n, n, n)
    L = 200.0
    return Problem("cgl3d_complex", shape, ("periodic",) * 3, (complex(1.0, CGL_ALPHA),), 0.05,
                   "cgl_z", {"beta": CGL_BETA}, nsteps, h=tuple(L / m for m in shape), seed=seed,
                   ic="gaussian_pulses", ic_args={"width": 1000.0, "c1": 50.0, "c2": 100.0})


def cgl2d_complex(n: int = 400, nsteps: int = 200, seed: int = 0) -> Problem:
    """Complex Ginzburg-Landau on the periodic square [0, 200]^2 at Section
    8.3's 2-D size (p = 400, h = 1/2, k = 1/20, beta = 1.3, its three
    Gaussian pulses), with alpha = 0.5."""
    L = 200.0
    return Problem("cgl2d_complex", (n, n), ("periodic",) * 2, (complex(1.0, CGL_ALPHA),), 0.05,
                   "cgl_z", {"beta": CGL_BETA}, nsteps, h=(L / n, L / n), seed=seed,
                   ic="gaussian_pulses_2d", ic_args={"width": 1000.0})


@dataclass
class Ensemble:
    """A batch of independent 2-D problems (one reaction model, one k)."""
    name: str
    model: str
    k: float
    nsteps: int
    instances: list          # dicts: shape, bcs, D, params
    states: list             # initial states, (s, n_2, n_1) each

    @property
    def s(self) -> int:
        return len(self.instances[0]["D"])

    @property
    def cell_species(self) -> int:
        return sum(ins["shape"][0] * ins["shape"][1] for ins in self.instances) * self.s


def brusselator_ensemble(ninst: int = 1024, nsteps: int = 200, seed: int = 0,
                         sizes=tuple(range(64, 513, 32))) -> Ensemble:
    """Independent 2-D Brusselators (a = 1): per instance, in draw order,
    N ~ U(sizes), b ~ U[2, 4], D1, D2 ~ U[1e-3, 5e-2], bc_x, bc_y ~
    U{Neumann, periodic}; square N x N grids on the unit square; initial data
    0.5 + 0.1 U[0, 1) per cell and species; k = 0.005."""
    rng = np.random.default_rng(seed)
    insts = []
    for _ in range(ninst):
        n = int(rng.choice(np.asarray(sizes)))
        b = float(rng.uniform(2.0, 4.0))
        d1 = float(rng.uniform(1e-3, 5e-2))
        d2 = float(rng.uniform(1e-3, 5e-2))
        bcs = tuple("neumann" if rng.integers(2) == 0 else "periodic" for _ in range(2))
        insts.append({"shape": (n, n), "bcs": bcs, "D": (d1, d2), "params": {"a": 1.0, "b": b}})
    states = [np.stack([0.5 + 0.1 * rng.random((ins["shape"][1], ins["shape"][0])) for _ in range(2)])
              for ins in insts]
    return Ensemble("brusselator_ensemble", "brusselator", 0.005, nsteps, insts, states)


WORKLOADS = {
    "brusselator2d": brusselator2d,
    "grayscott3d": grayscott3d,
    "grayscott4d": grayscott4d,
    "grayscott5d": grayscott5d,
    "schnakenberg3d": schnakenberg3d,
    "schnakenberg3d_adjoint": schnakenberg3d_adjoint,
    "cgl3d_complex": cgl3d_complex,
    "cgl2d_complex": cgl2d_complex,
}
