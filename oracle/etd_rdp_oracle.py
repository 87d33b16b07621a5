"""Plain FP64 reference of the ETD-RDP-IF time step.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing outside
``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may use this module.

Array convention.  A state with ``s`` species on a ``d``-dimensional grid is a
numpy array of shape ``(s, n_d, ..., n_2, n_1)``: species slowest, spatial axis
1 fastest.  Spatial axis ``i`` (1-based, as in the paper's ``A_i``) is numpy
axis ``d - i + 1``.  This matches the Kronecker order of Example 2 (Section 3),
where ``B_p`` of ``A_1`` sits in the innermost spatial position and ``B_p`` of
``A_d`` in the outermost one; the paper additionally puts the species index
innermost, which is only a permutation of the same vector.

Line solves.  Each split operator ``(I + (k/gamma) A_i)`` acts on the grid as an
independent 1-D solve along axis ``i`` with the per-species matrix
``I + (k/gamma) D_sigma B_p`` (Section 7).  Homogeneous Dirichlet and Neumann
lines are solved with LAPACK's banded Gaussian elimination
(``scipy.linalg.solve_banded``); periodic lines are circulant and are solved
by diagonalisation with the FFT, the route Section 7 itself describes.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg

BC_DIRICHLET = "dirichlet"
BC_NEUMANN = "neumann"
BC_PERIODIC = "periodic"
_BCS = (BC_DIRICHLET, BC_NEUMANN, BC_PERIODIC)


# ---------------------------------------------------------------------------
# Space discretisation (Section 3, Example 1 and Example 2)
# ---------------------------------------------------------------------------

def default_h(n: int, bc: str) -> float:
    """Grid spacing on the unit interval for ``n`` unknowns (Example 1):
    Dirichlet ``1/(n+1)``, Neumann ``1/(n-1)``, periodic ``1/n``."""
    if bc == BC_DIRICHLET:
        return 1.0 / (n + 1)
    if bc == BC_NEUMANN:
        return 1.0 / (n - 1)
    if bc == BC_PERIODIC:
        return 1.0 / n
    raise ValueError(bc)


def laplacian_matrix(n: int, bc: str, h: float) -> np.ndarray:
    """Dense ``B_p`` of Example 1: the centred second difference of ``-u''``.

    Interior rows are ``(-1, 2, -1)/h^2``.  Neumann replaces the first row's
    super-diagonal and the last row's sub-diagonal by ``-2/h^2`` (reflected
    ghost values), so the matrix is not symmetric.  Periodic adds ``-1/h^2``
    in the two corners.
    """
    if bc not in _BCS:
        raise ValueError(bc)
    B = np.zeros((n, n))
    for j in range(n):
        B[j, j] = 2.0
        if j > 0:
            B[j, j - 1] = -1.0
        if j < n - 1:
            B[j, j + 1] = -1.0
    if bc == BC_NEUMANN:
        B[0, 1] = -2.0
        B[n - 1, n - 2] = -2.0
    elif bc == BC_PERIODIC:
        B[0, n - 1] += -1.0
        B[n - 1, 0] += -1.0
    return B / (h * h)


def line_matrix(n: int, bc: str, h: float, coef: float) -> np.ndarray:
    """Dense ``I + coef * B_p``: one line of ``I + (k/gamma) A_i`` for one
    species, with ``coef = k D_sigma / gamma`` (Section 7)."""
    return np.eye(n) + coef * laplacian_matrix(n, bc, h)


def _solve_lines(n: int, bc: str, h: float, coef: float, rhs: np.ndarray) -> np.ndarray:
    """Solve ``(I + coef B_p) X = rhs`` for every column of ``rhs`` (n, m)."""
    if coef == 0.0:
        return rhs.copy()
    if bc == BC_PERIODIC:
        # Circulant: first column (1 + 2rho, -rho, 0, ..., 0, -rho); its
        # eigenvalues are the DFT of that column (Section 7).
        col = np.zeros(n)
        col[0] = 1.0
        col += coef * laplacian_matrix(n, bc, h)[:, 0]
        lam = np.fft.fft(col)
        return np.real(np.fft.ifft(np.fft.fft(rhs, axis=0) / lam[:, None], axis=0))
    M = line_matrix(n, bc, h, coef)
    ab = np.zeros((3, n))
    ab[0, 1:] = np.diag(M, 1)
    ab[1, :] = np.diag(M)
    ab[2, :-1] = np.diag(M, -1)
    return scipy.linalg.solve_banded((1, 1), ab, rhs)


def solve_axis(U: np.ndarray, axis: int, coefs, bc: str, h: float) -> np.ndarray:
    """Apply ``(I + (k/gamma) A_axis)^{-1}`` to a state ``U`` of shape
    ``(s, n_d, ..., n_1)``: a 1-D solve along spatial ``axis`` (1-based) for
    every grid line and species, species ``sigma`` using ``coefs[sigma]``."""
    d = U.ndim - 1
    npax = d - axis + 1
    out = np.empty_like(U)
    n = U.shape[npax]
    for sigma in range(U.shape[0]):
        X = np.moveaxis(U[sigma], npax - 1, 0)
        shp = X.shape
        Y = _solve_lines(n, bc, h, float(coefs[sigma]), X.reshape(n, -1))
        out[sigma] = np.moveaxis(Y.reshape(shp), 0, npax - 1)
    return out


def apply_R(U, axis, k, D, bc, h):
    """``R_RDP(k A_axis) U = 9 T U - 8 S U`` with ``T = (I + k/3 A)^{-1}`` and
    ``S = (I + k/4 A)^{-1}`` (partial fractions of Section 6)."""
    D = np.asarray(D, dtype=np.float64)
    T = solve_axis(U, axis, k * D / 3.0, bc, h)
    S = solve_axis(U, axis, k * D / 4.0, bc, h)
    return 9.0 * T - 8.0 * S


# ---------------------------------------------------------------------------
# Rational approximations of exp(-z) (Section 6)
# ---------------------------------------------------------------------------

def r_rdp(z):
    """``R_RDP(z) = (1 - 5z/12) / ((1 + z/3)(1 + z/4))`` (eq. padenonlinear)."""
    z = np.asarray(z, dtype=np.float64)
    return (1.0 - 5.0 * z / 12.0) / ((1.0 + z / 3.0) * (1.0 + z / 4.0))


def r_pade01(z):
    """``R_01(z) = 1/(1 + z)`` (eq. pade01)."""
    z = np.asarray(z, dtype=np.float64)
    return 1.0 / (1.0 + z)


# ---------------------------------------------------------------------------
# Reactions F(u) (Section 8 workloads and the benchmark systems)
# ---------------------------------------------------------------------------

def reaction(model: str, params: dict, U: np.ndarray) -> np.ndarray:
    """Pointwise reaction ``F(U)`` for a state of shape ``(s, ...)``.

    ``params['shift']`` (optional, one value per species) evaluates F at
    ``U + shift``; it turns a steady state ``u*`` into the origin so that a
    homogeneous Dirichlet condition can be posed on ``u - u*``.
    """
    shift = params.get("shift")
    if shift is not None:
        U = U + np.asarray(shift, dtype=np.float64).reshape((-1,) + (1,) * (U.ndim - 1))
    if model == "linear":
        # F(u) = C u, C an s x s constant matrix.
        C = np.atleast_2d(np.asarray(params["C"], dtype=np.float64))
        return np.tensordot(C, U, axes=(1, 0))
    if model == "enzyme":
        # Michaelis-Menten enzyme kinetics, s = 1: f = -u/(1+u) (Section 8.1).
        return -U / (1.0 + U)
    if model == "brusselator":
        # u' = a - (b+1) u + u^2 v,  v' = b u - u^2 v  (Section 8.2 with the
        # paper's A = b and B = a).
        a, b = params["a"], params["b"]
        u, v = U[0], U[1]
        uuv = u * u * v
        return np.stack([a - (b + 1.0) * u + uuv, b * u - uuv])
    if model == "gray_scott":
        # u' = -u v^2 + F (1 - u),  v' = u v^2 - (F + kappa) v.
        F, kap = params["F"], params["kappa"]
        u, v = U[0], U[1]
        uvv = u * v * v
        return np.stack([-uvv + F * (1.0 - u), uvv - (F + kap) * v])
    if model == "schnakenberg":
        # u' = gamma (a - u + u^2 v),  v' = gamma (b - u^2 v).
        a, b, g = params["a"], params["b"], params["gamma"]
        u, v = U[0], U[1]
        uuv = u * u * v
        return np.stack([g * (a - u + uuv), g * (b - uuv)])
    if model == "cgl":
        # Complex Ginzburg-Landau with alpha = 0 written for (Re u, Im u)
        # (Section 8.3): f = u - (1 + i beta) u |u|^2.
        beta = params["beta"]
        p, q = U[0], U[1]
        m2 = p * p + q * q
        return np.stack([p - (p - beta * q) * m2, q - (q + beta * p) * m2])
    raise ValueError(model)


# ---------------------------------------------------------------------------
# The ETD-RDP-IF step (Section 6, eq. donedone and the d-dimensional frame)
# ---------------------------------------------------------------------------

def _check(U, D, bcs, hs):
    d = U.ndim - 1
    if len(bcs) != d or len(hs) != d or len(D) != U.shape[0]:
        raise ValueError("shape/parameter mismatch")


def step_intermediates(U, k, D, bcs, hs, model, params):
    """One ETD-RDP-IF step with every intermediate returned.

    ``bcs[i-1]``, ``hs[i-1]`` describe spatial axis ``i``.  Follows the
    d-dimensional frame of Section 6:

    * predictor ``U* = (I+kA_d)^{-1} ... (I+kA_1)^{-1} (U_n + k f(U_n))``;
    * the factors ``{9 (I+k/3 A_i)^{-1} - 8 (I+k/4 A_i)^{-1}}`` for
      ``i = 1..d-1`` applied to ``U_n`` and to ``f(U_n)`` (linearity lets the
      two bracketed combinations ``9U+2kf`` and ``8U+3k/2 f`` be formed after
      the factors);
    * corrector ``U_{n+1} = (I+k/3 A_d)^{-1}[9 cU + 2k cf + k f*]
      - (I+k/4 A_d)^{-1}[8 cU + 3k/2 cf + k/2 f*]``.

    The corrector's second bracket carries all three terms with a minus sign,
    as in eq. donedone and the 2-D flow chart; the 3-D flow chart prints the
    first term of ``f_2`` with the opposite sign, which is taken as a misprint
    (with D = 0 only this reading reduces to Heun's method).
    """
    U = np.asarray(U, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    _check(U, D, bcs, hs)
    d = U.ndim - 1
    out = {}
    f = reaction(model, params, U)
    out["f"] = f
    y = U + k * f
    out["w"] = y
    for i in range(1, d + 1):
        y = solve_axis(y, i, k * D, bcs[i - 1], hs[i - 1])
        out[f"y{i}"] = y
    Ustar = y
    out["Ustar"] = Ustar
    cU, cf = U, f
    for i in range(1, d):
        cU = apply_R(cU, i, k, D, bcs[i - 1], hs[i - 1])
        cf = apply_R(cf, i, k, D, bcs[i - 1], hs[i - 1])
        out[f"cU{i}"] = cU
        out[f"cf{i}"] = cf
    fstar = reaction(model, params, Ustar)
    out["fstar"] = fstar
    f1 = 9.0 * cU + 2.0 * k * cf + k * fstar
    f2 = 8.0 * cU + 1.5 * k * cf + 0.5 * k * fstar
    out["f1"], out["f2"] = f1, f2
    bd, hd = bcs[d - 1], hs[d - 1]
    d1 = solve_axis(f1, d, k * D / 3.0, bd, hd)
    d2 = solve_axis(f2, d, k * D / 4.0, bd, hd)
    out["Unew"] = d1 - d2
    return out


def etd_rdp_if_step(U, k, D, bcs, hs, model, params):
    """``U_{n+1}`` from ``U_n`` (see :func:`step_intermediates`)."""
    return step_intermediates(U, k, D, bcs, hs, model, params)["Unew"]


def etd_rdp_if_run(U, k, D, bcs, hs, model, params, nsteps):
    """``nsteps`` steps of the scheme (the time loop of the frame)."""
    for _ in range(int(nsteps)):
        U = etd_rdp_if_step(U, k, D, bcs, hs, model, params)
    return U


def etd1_if_step(U, k, D, bcs, hs, model, params):
    """First-order predictor alone (ETD1 = IMEX backward Euler with the same
    integrating-factor splitting, eq. duhamel3t with the Pade-(0,1) factor)."""
    U = np.asarray(U, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    _check(U, D, bcs, hs)
    y = U + k * reaction(model, params, U)
    for i in range(1, U.ndim):
        y = solve_axis(y, i, k * D, bcs[i - 1], hs[i - 1])
    return y
