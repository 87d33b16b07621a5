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

Complex species.  A complex scalar diffusion coefficient (the complex
Ginzburg-Landau equation with alpha != 0, and the cubic Schroedinger
equation, Section 8.3 and 8.4) is handled by the same functions with complex
arrays: a complex state of shape ``(s, n_d, ..., n_1)`` and complex ``D``.
The line systems ``I + (k/gamma) D_sigma B_p`` are then complex tridiagonal
(or circulant), solved by the same banded elimination or FFT.
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


def _solve_lines(n: int, bc: str, h: float, coef, rhs: np.ndarray) -> np.ndarray:
    """Solve ``(I + coef B_p) X = rhs`` for every column of ``rhs`` (n, m);
    ``coef`` and ``rhs`` may be complex."""
    if coef == 0.0:
        return rhs.copy()
    real = not (np.iscomplexobj(rhs) or isinstance(coef, complex))
    if bc == BC_PERIODIC:
        # Circulant: first column (1 + 2rho, -rho, 0, ..., 0, -rho); its
        # eigenvalues are the DFT of that column (Section 7).
        col = np.zeros(n, dtype=np.float64 if real else np.complex128)
        col[0] = 1.0
        col += coef * laplacian_matrix(n, bc, h)[:, 0]
        lam = np.fft.fft(col)
        X = np.fft.ifft(np.fft.fft(rhs, axis=0) / lam[:, None], axis=0)
        return np.real(X) if real else X
    M = line_matrix(n, bc, h, coef)
    ab = np.zeros((3, n), dtype=M.dtype)
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
    cplx = np.iscomplexobj(U) or np.iscomplexobj(coefs)
    out = np.empty(U.shape, dtype=np.complex128 if cplx else np.float64)
    n = U.shape[npax]
    for sigma in range(U.shape[0]):
        X = np.moveaxis(U[sigma], npax - 1, 0)
        shp = X.shape
        cf = complex(coefs[sigma]) if cplx else float(coefs[sigma])
        Y = _solve_lines(n, bc, h, cf, X.reshape(n, -1))
        out[sigma] = np.moveaxis(Y.reshape(shp), 0, npax - 1)
    return out


def apply_R(U, axis, k, D, bc, h):
    """``R_RDP(k A_axis) U = 9 T U - 8 S U`` with ``T = (I + k/3 A)^{-1}`` and
    ``S = (I + k/4 A)^{-1}`` (partial fractions of Section 6)."""
    D = _coefs(D)
    T = solve_axis(U, axis, k * D / 3.0, bc, h)
    S = solve_axis(U, axis, k * D / 4.0, bc, h)
    return 9.0 * T - 8.0 * S


# ---------------------------------------------------------------------------
# Rational approximations of exp(-z) (Section 6)
# ---------------------------------------------------------------------------

def r_rdp(z):
    """``R_RDP(z) = (1 - 5z/12) / ((1 + z/3)(1 + z/4))`` (eq. padenonlinear)."""
    z = _coefs(z)
    return (1.0 - 5.0 * z / 12.0) / ((1.0 + z / 3.0) * (1.0 + z / 4.0))


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
    if model == "cgl_z":
        # Complex Ginzburg-Landau for a complex state, s = 1 (Section 8.3):
        # f = u - (1 + i beta) u |u|^2; alpha enters through D = 1 + i alpha.
        beta = params["beta"]
        u = U
        return u - (1.0 + 1j * beta) * u * (u * np.conj(u)).real
    if model == "nls_z":
        # Cubic Schroedinger equation i psi_t + Lap psi = q psi with
        # q = B + C |psi|^2, written as psi_t = i Lap psi - i q psi
        # (D = i, Section 8.4).  An optional per-cell field (params["Bfield"],
        # shaped like one species) is added to the constant B: the spatially
        # varying B(x, y) of the 2-D example.
        B, C = params["B"], params["C"]
        Bf = params.get("Bfield")
        q = B + C * (U * np.conj(U)).real
        if Bf is not None:
            q = q + np.asarray(Bf, dtype=np.float64)
        return -1j * q * U
    raise ValueError(model)


# ---------------------------------------------------------------------------
# The ETD-RDP-IF step (Section 6, eq. donedone and the d-dimensional frame)
# ---------------------------------------------------------------------------

def _coefs(D):
    """Diffusion coefficients as a float64 array, or complex128 when any is
    complex."""
    D = np.asarray(D)
    return D.astype(np.complex128) if np.iscomplexobj(D) else D.astype(np.float64)


def _state(U):
    U = np.asarray(U)
    return U.astype(np.complex128) if np.iscomplexobj(U) else U.astype(np.float64)


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
    U = _state(U)
    D = _coefs(D)
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
    U = _state(U)
    D = _coefs(D)
    _check(U, D, bcs, hs)
    y = U + k * reaction(model, params, U)
    for i in range(1, U.ndim):
        y = solve_axis(y, i, k * D, bcs[i - 1], hs[i - 1])
    return y


# ---------------------------------------------------------------------------
# Reverse mode of one step (not in the paper: the chain rule applied to the
# frame of Section 6, used to check the GPU adjoint)
# ---------------------------------------------------------------------------

MODEL_PARAM_NAMES = {"enzyme": (), "brusselator": ("a", "b"), "gray_scott": ("F", "kappa"),
                     "schnakenberg": ("a", "b", "gamma"), "cgl": ("beta",)}


def param_names(model, s):
    if model == "linear":
        return tuple(f"C{i}{j}" for i in range(s) for j in range(s))
    return MODEL_PARAM_NAMES[model]


def reaction_jacobian(model, params, U):
    """J[i][j] = dF_i/du_j at every cell (arrays shaped like U[0])."""
    shift = params.get("shift")
    if shift is not None:
        U = U + np.asarray(shift, dtype=np.float64).reshape((-1,) + (1,) * (U.ndim - 1))
    one = np.ones_like(U[0])
    if model == "linear":
        C = np.atleast_2d(np.asarray(params["C"], dtype=np.float64))
        s = C.shape[0]
        return [[C[i, j] * one for j in range(s)] for i in range(s)]
    if model == "enzyme":
        return [[-1.0 / (1.0 + U[0]) ** 2]]
    u, v = U[0], U[1]
    if model == "brusselator":
        b = params["b"]
        return [[-(b + 1.0) + 2 * u * v, u * u], [b - 2 * u * v, -u * u]]
    if model == "gray_scott":
        F, kap = params["F"], params["kappa"]
        return [[-v * v - F, -2 * u * v], [v * v, 2 * u * v - (F + kap)]]
    if model == "schnakenberg":
        g = params["gamma"]
        return [[g * (-1.0 + 2 * u * v), g * u * u], [-2 * g * u * v, -g * u * u]]
    if model == "cgl":
        beta = params["beta"]
        p, q = u, v
        m2 = p * p + q * q
        return [[1 - m2 - 2 * p * (p - beta * q), beta * m2 - 2 * q * (p - beta * q)],
                [-beta * m2 - 2 * p * (q + beta * p), 1 - m2 - 2 * q * (q + beta * p)]]
    raise ValueError(model)


def reaction_param_grads(model, params, U):
    """dF/dtheta for each model parameter: a list (over parameters) of
    arrays shaped like U."""
    shift = params.get("shift")
    if shift is not None:
        U = U + np.asarray(shift, dtype=np.float64).reshape((-1,) + (1,) * (U.ndim - 1))
    z = np.zeros_like(U[0])
    one = np.ones_like(U[0])
    if model == "linear":
        s = U.shape[0]
        out = []
        for i in range(s):
            for j in range(s):
                g = np.zeros_like(U)
                g[i] = U[j]
                out.append(g)
        return out
    if model == "enzyme":
        return []
    u, v = U[0], U[1]
    if model == "brusselator":
        return [np.stack([one, z]), np.stack([-u, u])]
    if model == "gray_scott":
        return [np.stack([1.0 - u, -v]), np.stack([z, -v])]
    if model == "schnakenberg":
        a, b, g = params["a"], params["b"], params["gamma"]
        return [np.stack([g * one, z]), np.stack([z, g * one]),
                np.stack([a - u + u * u * v, b - u * u * v])]
    if model == "cgl":
        m2 = u * u + v * v
        return [np.stack([v * m2, -u * m2])]
    raise ValueError(model)


def _jac_T(J, w):
    s = len(J)
    return np.stack([sum(J[i][j] * w[i] for i in range(s)) for j in range(s)])


def solve_axis_T(U, axis, coefs, bc, h):
    """Apply (I + c B_p)^{-T} along `axis` (dense transposed solve per species)."""
    d = U.ndim - 1
    npax = d - axis + 1
    out = np.empty_like(U)
    n = U.shape[npax]
    for sigma in range(U.shape[0]):
        M = line_matrix(n, bc, h, float(coefs[sigma]))
        X = np.moveaxis(U[sigma], npax - 1, 0)
        shp = X.shape
        Y = np.linalg.solve(M.T, X.reshape(n, -1))
        out[sigma] = np.moveaxis(Y.reshape(shp), 0, npax - 1)
    return out


def laplacian_axis(U, axis, bc, h):
    """B_p (the discrete -Laplacian of Example 1) applied along `axis`."""
    d = U.ndim - 1
    npax = d - axis + 1
    n = U.shape[npax]
    B = laplacian_matrix(n, bc, h)
    out = np.empty_like(U)
    for sigma in range(U.shape[0]):
        X = np.moveaxis(U[sigma], npax - 1, 0)
        shp = X.shape
        out[sigma] = np.moveaxis((B @ X.reshape(n, -1)).reshape(shp), 0, npax - 1)
    return out


def adjoint_step(U, lam, k, D, bcs, hs, model, params, term_scale=None):
    """Vector-Jacobian product of one ETD-RDP-IF step.

    Given U_n and lam = dL/dU_{n+1}, returns (dL/dU_n, dL/dD, dL/dtheta) for
    this step, where theta are the reaction parameters (``param_names``).
    A solve x = M^{-1} y with M = I + (k/gamma) D_sigma B_p contributes
    -(k/gamma) <M^{-T} xbar, B_p x>_sigma to dL/dD_sigma.

    ``term_scale``: optional dict that receives, under "D" and "theta", the
    sum of the absolute values of every per-cell term added into each
    gradient entry (the size of the terms before they cancel; a diagnostic
    for judging how many digits of an entry rounding leaves).
    """
    U = np.asarray(U, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    d = U.ndim - 1
    s = U.shape[0]
    gD = np.zeros(s)
    gth = np.zeros(len(param_names(model, s)))
    sD = np.zeros(s)
    sth = np.zeros(len(gth))

    def dgrad(ybar, x, axis, gamma):
        Lx = laplacian_axis(x, axis, bcs[axis - 1], hs[axis - 1])
        for sg in range(s):
            gD[sg] += -(k / gamma) * float(np.sum(ybar[sg] * Lx[sg]))
            sD[sg] += (k / gamma) * float(np.sum(np.abs(ybar[sg] * Lx[sg])))

    def pgrad(Uat, fbar):
        for i, dF in enumerate(reaction_param_grads(model, params, Uat)):
            gth[i] += float(np.sum(dF * fbar))
            sth[i] += float(np.sum(np.abs(dF * fbar)))

    # forward recomputation
    f = reaction(model, params, U)
    ys = [U + k * f]
    for i in range(1, d + 1):
        ys.append(solve_axis(ys[-1], i, k * D, bcs[i - 1], hs[i - 1]))
    Ustar = ys[d]
    cU, cf = [U], [f]
    for i in range(1, d):
        cU.append(apply_R(cU[-1], i, k, D, bcs[i - 1], hs[i - 1]))
        cf.append(apply_R(cf[-1], i, k, D, bcs[i - 1], hs[i - 1]))
    fs = reaction(model, params, Ustar)
    f1 = 9.0 * cU[-1] + 2.0 * k * cf[-1] + k * fs
    f2 = 8.0 * cU[-1] + 1.5 * k * cf[-1] + 0.5 * k * fs
    bd, hd = bcs[d - 1], hs[d - 1]
    # reverse: U_{n+1} = T_d f1 - S_d f2
    a = solve_axis_T(lam, d, k * D / 3.0, bd, hd)
    b = solve_axis_T(lam, d, k * D / 4.0, bd, hd)
    dgrad(a, solve_axis(f1, d, k * D / 3.0, bd, hd), d, 3.0)
    dgrad(-b, solve_axis(f2, d, k * D / 4.0, bd, hd), d, 4.0)
    fsbar = k * a - 0.5 * k * b
    pgrad(Ustar, fsbar)
    ybar = _jac_T(reaction_jacobian(model, params, Ustar), fsbar)
    cUbar = 9.0 * a - 8.0 * b
    cfbar = 2.0 * k * a - 1.5 * k * b
    for i in range(d, 0, -1):  # predictor chain P_d ... P_1
        yin = solve_axis_T(ybar, i, k * D, bcs[i - 1], hs[i - 1])
        dgrad(yin, ys[i], i, 1.0)
        ybar = yin
    nu = ybar
    for i in range(d - 1, 0, -1):  # R chains, R_i = 9 T_i - 8 S_i
        bc_, h_ = bcs[i - 1], hs[i - 1]
        nxt = []
        for cbar, cin in ((cUbar, cU[i - 1]), (cfbar, cf[i - 1])):
            tb = solve_axis_T(9.0 * cbar, i, k * D / 3.0, bc_, h_)
            sb = solve_axis_T(-8.0 * cbar, i, k * D / 4.0, bc_, h_)
            dgrad(tb, solve_axis(cin, i, k * D / 3.0, bc_, h_), i, 3.0)
            dgrad(sb, solve_axis(cin, i, k * D / 4.0, bc_, h_), i, 4.0)
            nxt.append(tb + sb)
        cUbar, cfbar = nxt
    fbar = cfbar + k * nu
    pgrad(U, fbar)
    lam_n = cUbar + nu + _jac_T(reaction_jacobian(model, params, U), fbar)
    if term_scale is not None:
        term_scale["D"] = sD
        term_scale["theta"] = sth
    return lam_n, gD, gth
