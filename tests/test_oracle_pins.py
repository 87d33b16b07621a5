"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here uses something other than the oracle's own formulas:
closed-form eigenpairs of the paper's B_p matrices, the closed form of the
rational approximation, dense Kronecker matrices built from Example 2,
the exact solution of linear problems, invariants and observed convergence.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
BCS = (O.BC_DIRICHLET, O.BC_NEUMANN, O.BC_PERIODIC)


# ---------------------------------------------------------------------------
# B_p eigenpairs (Example 1): eigenvectors in closed form
# ---------------------------------------------------------------------------

def _mode(n, bc, j):
    """Closed-form eigenvector and eigenvalue of B_p (unit interval)."""
    h = O.default_h(n, bc)
    m = np.arange(n)
    if bc == O.BC_DIRICHLET:
        x = (m + 1) * h
        v = np.sin(j * math.pi * x)
        lam = 4.0 / h**2 * math.sin(j * math.pi * h / 2) ** 2
    elif bc == O.BC_NEUMANN:
        x = m * h
        v = np.cos(j * math.pi * x)
        lam = 4.0 / h**2 * math.sin(j * math.pi * h / 2) ** 2
    else:
        v = np.cos(2 * math.pi * j * m / n)
        lam = 4.0 / h**2 * math.sin(math.pi * j / n) ** 2
    return v, lam, h


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", [5, 8, 17])
def test_laplacian_eigenpairs(bc, n):
    for j in range(1, 4):
        v, lam, h = _mode(n, bc, j)
        B = O.laplacian_matrix(n, bc, h)
        np.testing.assert_allclose(B @ v, lam * v, rtol=0, atol=1e-10 * lam * np.abs(v).max() + 1e-12)


def test_neumann_left_null_vector():
    # Trapezoid weights annihilate the Neumann B_p from the left: the discrete
    # Neumann problem conserves the trapezoid-weighted total.
    for n in (2, 3, 9, 40):
        B = O.laplacian_matrix(n, O.BC_NEUMANN, 0.3)
        W = np.ones(n)
        W[0] = W[-1] = 0.5
        np.testing.assert_allclose(W @ B, 0.0, atol=1e-12)
    B = O.laplacian_matrix(7, O.BC_PERIODIC, 0.3)
    np.testing.assert_allclose(np.ones(7) @ B, 0.0, atol=1e-12)


@pytest.mark.parametrize("bc", BCS)
def test_solve_axis_matches_dense_solve(bc):
    rng = np.random.default_rng(1)
    U = rng.standard_normal((2, 4, 5, 6))
    coefs = np.array([0.37, 2.9])
    hs = [O.default_h(n, bc) for n in (6, 5, 4)]
    for axis in (1, 2, 3):
        n = U.shape[4 - axis]
        h = hs[axis - 1]
        X = O.solve_axis(U, axis, coefs, bc, h)
        for s in range(2):
            M = np.eye(n) + coefs[s] * O.laplacian_matrix(n, bc, h)
            A = np.moveaxis(U[s], 3 - axis, 0).reshape(n, -1)
            ref = np.linalg.solve(M, A)
            got = np.moveaxis(X[s], 3 - axis, 0).reshape(n, -1)
            np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------------------
# Rational approximation (Section 6): closed form, L-stability, order
# ---------------------------------------------------------------------------

def _one_d_mode_step(bc, n, j, z, nsteps=1, F=None):
    """One F = 0 step of the 1-D scheme on an eigenvector with k D lam = z."""
    v, lam, h = _mode(n, bc, j)
    k = 0.1
    D = z / (k * lam)
    U = v[None, :].copy()
    model, params = ("linear", {"C": [[0.0]]}) if F is None else F
    return O.etd_rdp_if_step(U, k, [D], [bc], [h], model, params)[0], v


@pytest.mark.parametrize("bc", BCS)
def test_F0_single_mode_is_rdp_closed_form(bc):
    num = GOLD["rdp_numerator_coef"]["value"]
    p1, p2 = GOLD["rdp_poles"]["value"]
    w1, w2 = GOLD["partial_fractions"]["value"]["R"]
    for z in (1e-3, 0.2, 1.0, 7.5, 300.0):
        got, v = _one_d_mode_step(bc, 12, 2, z)
        r = (1.0 - num * z) / ((1.0 + z / p1) * (1.0 + z / p2))
        np.testing.assert_allclose(got, r * v, rtol=1e-12, atol=1e-14)
        # the same number through the printed partial fractions 9T - 8S
        np.testing.assert_allclose(got, (w1 / (1.0 + z / p1) + w2 / (1.0 + z / p2)) * v,
                                   rtol=1e-12, atol=1e-14)


def test_partial_fraction_identities():
    """The three decompositions of Section 6, with the printed weights, hold as
    rational functions of z (T = 1/(1 + z/3), S = 1/(1 + z/4)):
    R_RDP = 9T - 8S, ST = 4T - 3S, (1 + z/6) ST = 2T - S."""
    pf = GOLD["partial_fractions"]["value"]
    p1, p2 = GOLD["rdp_poles"]["value"]
    num = GOLD["rdp_numerator_coef"]["value"]
    z = np.concatenate([np.linspace(0.0, 20.0, 401), np.logspace(1, 6, 50)])
    T, S = 1.0 / (1.0 + z / p1), 1.0 / (1.0 + z / p2)
    np.testing.assert_allclose(pf["R"][0] * T + pf["R"][1] * S, (1.0 - num * z) * S * T,
                               rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(pf["ST"][0] * T + pf["ST"][1] * S, S * T, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(pf["I_plus_k6A_ST"][0] * T + pf["I_plus_k6A_ST"][1] * S,
                               (1.0 + z / 6.0) * S * T, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(O.r_rdp(z), pf["R"][0] * T + pf["R"][1] * S, rtol=1e-12,
                               atol=1e-15)


def test_rdp_l_stability_and_order():
    z = np.concatenate([np.linspace(0, 10, 1001), np.logspace(1, 8, 200)])
    # The oracle applies 9T - 8S; evaluate it on a 1x1 system B = [lam].
    vals = []
    for zz in (0.0, 0.5, 3.0, 40.0, 1e4, 1e8):
        got, v = _one_d_mode_step(O.BC_DIRICHLET, 6, 1, zz)
        vals.append(got[0] / v[0])
    vals = np.array(vals)
    assert np.all(np.abs(vals) <= 1.0 + 1e-14)
    # z r(z) -> -5 as z -> infinity (L-stability: r(inf) = 0).
    assert abs(1e8 * vals[-1] + 5.0) < 1e-5
    # Local error r(z) - exp(-z) = -z^3/24 + O(z^4).
    for zz in (1e-2, 5e-3):
        got, v = _one_d_mode_step(O.BC_DIRICHLET, 6, 1, zz)
        err = got[0] / v[0] - math.exp(-zz)
        assert abs(err / zz**3 + 1.0 / 24.0) < 0.02
    # and the closed form itself never exceeds 1 in magnitude on z >= 0
    assert np.all(np.abs(O.r_rdp(z)) <= 1.0)


def test_predictor_is_pade01():
    # Pade-(0,1) of eq. pade01: 1/(1 + z/pole) with the printed pole 1
    pole = GOLD["pade01_pole"]["value"]
    for bc in BCS:
        v, lam, h = _mode(10, bc, 1)
        k = 0.1
        for z in (0.05, 2.5, 40.0):
            U = v[None, :]
            got = O.etd1_if_step(U, k, [z / (k * lam)], [bc], [h], "linear", {"C": [[0.0]]})[0]
            np.testing.assert_allclose(got, v / (1.0 + z / pole), rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------------------
# Whole step: dense Kronecker brute force (Example 2, eq. donedone)
# ---------------------------------------------------------------------------

def _dense_ops(U, D, bcs, hs):
    """Dense A_1..A_d of eq. Ai for a state shaped like U, and the maps
    between a state and the paper's vector (species index innermost, then
    spatial axis 1, ..., axis d outermost; A_i = I x .. x B_p (position
    d-i+1) x .. x I x D)."""
    s = U.shape[0]
    d = U.ndim - 1
    ns = [U.shape[d - i + 1] for i in range(1, d + 1)]  # n_1..n_d
    Dm = np.diag(D)
    A = []
    for i in range(1, d + 1):
        mats = []
        for pos in range(1, d + 1):  # Kronecker position 1 = outermost = axis d
            ax = d - pos + 1
            mats.append(O.laplacian_matrix(ns[ax - 1], bcs[ax - 1], hs[ax - 1]) if ax == i
                        else np.eye(ns[ax - 1]))
        K = mats[0]
        for M in mats[1:]:
            K = np.kron(K, M)
        A.append(np.kron(K, Dm))
    vec = lambda X: np.moveaxis(X, 0, -1).reshape(-1)
    unvec = lambda x: np.moveaxis(x.reshape(U.shape[1:] + (s,)), -1, 0)
    return A, vec, unvec


def test_step_intermediates_match_dense_operators():
    """Each intermediate the GPU passes are compared with is what its name
    says: y_i = (I + k A_i)^{-1} y_{i-1}, cU_i = (9 (I + k/3 A_i)^{-1}
    - 8 (I + k/4 A_i)^{-1}) cU_{i-1} (and cf_i likewise), f* = F(U*),
    f1 = 9 cU + 2k cf + k f*, f2 = 8 cU + 3k/2 cf + k/2 f*."""
    rng = np.random.default_rng(11)
    U = 0.5 + 0.3 * rng.random((2, 4, 3, 5))  # n_1 = 5, n_2 = 3, n_3 = 4
    bcs = (O.BC_PERIODIC, O.BC_NEUMANN, O.BC_DIRICHLET)
    hs = [O.default_h(n, b) for n, b in zip((5, 3, 4), bcs)]
    D, k = np.array([0.03, 0.011]), 0.07
    p = {"F": 0.04, "kappa": 0.06}
    out = O.step_intermediates(U, k, D, bcs, hs, "gray_scott", p)
    A, vec, unvec = _dense_ops(U, D, bcs, hs)
    I = np.eye(A[0].shape[0])
    sol = lambda g, i, x: unvec(np.linalg.solve(I + k / g * A[i - 1], vec(x)))
    tol = dict(rtol=1e-12, atol=1e-14)
    f = O.reaction("gray_scott", p, U)
    np.testing.assert_allclose(out["w"], U + k * f, **tol)
    y = U + k * f
    for i in (1, 2, 3):
        y = sol(1.0, i, y)
        np.testing.assert_allclose(out[f"y{i}"], y, **tol)
    np.testing.assert_allclose(out["Ustar"], y, **tol)
    cU, cf = U, f
    for i in (1, 2):
        cU = 9 * sol(3.0, i, cU) - 8 * sol(4.0, i, cU)
        cf = 9 * sol(3.0, i, cf) - 8 * sol(4.0, i, cf)
        np.testing.assert_allclose(out[f"cU{i}"], cU, **tol)
        np.testing.assert_allclose(out[f"cf{i}"], cf, **tol)
    fs = O.reaction("gray_scott", p, y)
    np.testing.assert_allclose(out["fstar"], fs, **tol)
    np.testing.assert_allclose(out["f1"], 9 * cU + 2 * k * cf + k * fs, **tol)
    np.testing.assert_allclose(out["f2"], 8 * cU + 1.5 * k * cf + 0.5 * k * fs, **tol)


def _dense_step(U, k, D, bcs, hs, model, params):
    """The frame of Section 6 with explicit dense matrices.

    Vector ordering is the paper's: species index innermost, then spatial
    axis 1, ..., axis d outermost, and A_i = I x .. x B_p (position d-i+1)
    x .. x I x D (eq. Ai).
    """
    s = U.shape[0]
    d = U.ndim - 1
    ns = [U.shape[d - i + 1] for i in range(1, d + 1)]  # n_1..n_d
    Dm = np.diag(D)
    A = []
    for i in range(1, d + 1):
        mats = []
        for pos in range(1, d + 1):  # Kronecker position 1 = outermost = axis d
            ax = d - pos + 1
            mats.append(O.laplacian_matrix(ns[ax - 1], bcs[ax - 1], hs[ax - 1]) if ax == i
                        else np.eye(ns[ax - 1]))
        K = mats[0]
        for M in mats[1:]:
            K = np.kron(K, M)
        A.append(np.kron(K, Dm))
    m = A[0].shape[0]
    I = np.eye(m)
    vec = lambda X: np.moveaxis(X, 0, -1).reshape(-1)
    unvec = lambda x: np.moveaxis(x.reshape(U.shape[1:] + (s,)), -1, 0)
    f = lambda x: vec(O.reaction(model, params, unvec(x)))
    u = vec(U)
    fu = f(u)
    ustar = u + k * fu
    for i in range(d):
        ustar = np.linalg.solve(I + k * A[i], ustar)
    def Rfac(x):
        for i in range(d - 1):
            x = 9 * np.linalg.solve(I + k / 3 * A[i], x) - 8 * np.linalg.solve(I + k / 4 * A[i], x)
        return x
    fs = f(ustar)
    t1 = Rfac(9 * u + 2 * k * fu) + k * fs
    t2 = Rfac(8 * u + 1.5 * k * fu) + 0.5 * k * fs
    un = np.linalg.solve(I + k / 3 * A[d - 1], t1) - np.linalg.solve(I + k / 4 * A[d - 1], t2)
    return unvec(un)


@pytest.mark.parametrize("bcs", [
    (O.BC_DIRICHLET,) * 3, (O.BC_NEUMANN,) * 3, (O.BC_PERIODIC,) * 3,
    (O.BC_NEUMANN, O.BC_PERIODIC, O.BC_DIRICHLET), (O.BC_PERIODIC, O.BC_DIRICHLET, O.BC_NEUMANN),
])
def test_step_equals_dense_kronecker_3d(bcs):
    rng = np.random.default_rng(7)
    U = 0.5 + 0.3 * rng.random((2, 4, 5, 3))  # n_1 = 3, n_2 = 5, n_3 = 4
    ns = (3, 5, 4)
    hs = [O.default_h(n, b) for n, b in zip(ns, bcs)]
    D = [0.02, 0.011]
    for model, params in (("brusselator", {"a": 1.0, "b": 3.4}),
                          ("gray_scott", {"F": 0.04, "kappa": 0.06})):
        got = O.etd_rdp_if_step(U, 0.05, D, bcs, hs, model, params)
        ref = _dense_step(U, 0.05, np.array(D), bcs, hs, model, params)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("bcs", [
    (O.BC_NEUMANN, O.BC_PERIODIC, O.BC_DIRICHLET, O.BC_NEUMANN),
    (O.BC_PERIODIC, O.BC_DIRICHLET, O.BC_NEUMANN, O.BC_PERIODIC),
])
def test_step_equals_dense_kronecker_4d(bcs):
    # the general-d frame of Section 6 (four split factors, R on axes 1..3)
    rng = np.random.default_rng(9)
    U = 0.5 + 0.3 * rng.random((2, 3, 4, 2, 3))  # n_1 = 3, n_2 = 2, n_3 = 4, n_4 = 3
    ns = (3, 2, 4, 3)
    bcs = tuple(b if not (b == O.BC_PERIODIC and n < 3) else O.BC_NEUMANN for b, n in zip(bcs, ns))
    hs = [O.default_h(n, b) for n, b in zip(ns, bcs)]
    D = [0.02, 0.011]
    got = O.etd_rdp_if_step(U, 0.05, D, bcs, hs, "brusselator", {"a": 1.0, "b": 3.4})
    ref = _dense_step(U, 0.05, np.array(D), bcs, hs, "brusselator", {"a": 1.0, "b": 3.4})
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("bcs", [
    (O.BC_NEUMANN, O.BC_PERIODIC, O.BC_DIRICHLET, O.BC_NEUMANN, O.BC_PERIODIC),
    (O.BC_PERIODIC, O.BC_DIRICHLET, O.BC_NEUMANN, O.BC_PERIODIC, O.BC_DIRICHLET),
])
def test_step_equals_dense_kronecker_5d(bcs):
    # the general-d frame with five split factors (R on axes 1..4)
    rng = np.random.default_rng(10)
    ns = (3, 2, 3, 2, 3)  # n_1 .. n_5
    bcs = tuple(b if not (b == O.BC_PERIODIC and n < 3) else O.BC_NEUMANN for b, n in zip(bcs, ns))
    U = 0.5 + 0.3 * rng.random((2,) + ns[::-1])
    hs = [O.default_h(n, b) for n, b in zip(ns, bcs)]
    D = [0.02, 0.011]
    got = O.etd_rdp_if_step(U, 0.05, D, bcs, hs, "brusselator", {"a": 1.0, "b": 3.4})
    ref = _dense_step(U, 0.05, np.array(D), bcs, hs, "brusselator", {"a": 1.0, "b": 3.4})
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("bcs", [(O.BC_NEUMANN,) * 2, (O.BC_DIRICHLET, O.BC_PERIODIC)])
def test_step_equals_dense_kronecker_2d(bcs):
    rng = np.random.default_rng(8)
    U = rng.random((2, 6, 5))
    hs = [O.default_h(n, b) for n, b in zip((5, 6), bcs)]
    got = O.etd_rdp_if_step(U, 0.1, [0.3, 0.05], bcs, hs, "schnakenberg",
                            {"a": 0.1, "b": 0.9, "gamma": 1.0})
    ref = _dense_step(U, 0.1, np.array([0.3, 0.05]), bcs, hs, "schnakenberg",
                      {"a": 0.1, "b": 0.9, "gamma": 1.0})
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------------------
# Special cases that reduce to textbook schemes
# ---------------------------------------------------------------------------

def test_zero_diffusion_is_heun():
    rng = np.random.default_rng(3)
    U = 0.2 + rng.random((2, 4, 6, 5))
    bcs = (O.BC_NEUMANN, O.BC_PERIODIC, O.BC_DIRICHLET)
    hs = [0.1, 0.2, 0.3]
    k = 0.07
    p = {"a": 1.0, "b": 3.4}
    F = lambda X: O.reaction("brusselator", p, X)
    heun = U + 0.5 * k * (F(U) + F(U + k * F(U)))
    got = O.etd_rdp_if_step(U, k, [0.0, 0.0], bcs, hs, "brusselator", p)
    np.testing.assert_allclose(got, heun, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6])
def test_F0_separable_mode_is_product_of_r(d):
    bcs = [O.BC_DIRICHLET, O.BC_NEUMANN, O.BC_PERIODIC, O.BC_NEUMANN, O.BC_PERIODIC, O.BC_DIRICHLET][:d]
    ns = [7, 9, 8, 5, 6, 4][:d]
    js = [2, 1, 3, 2, 1, 3][:d]
    k, D = 0.05, [0.8]
    vs, lams, hs = zip(*[_mode(n, b, j) for n, b, j in zip(ns, bcs, js)])
    U = vs[0]
    for v in vs[1:]:
        U = np.multiply.outer(v, U)  # axis i+1 outermost
    U = U[None]
    got = O.etd_rdp_if_step(U, k, D, bcs, hs, "linear", {"C": [[0.0]]})
    g = np.prod([O.r_rdp(k * D[0] * lam) for lam in lams])
    np.testing.assert_allclose(got, g * U, rtol=1e-12, atol=1e-14)


def test_linear_reaction_converges_second_order_to_exact_mode():
    """F = c u on one separable mode: the exact solution is
    exp((c - D sum(lam)) t) times the mode; the scheme converges at order 2."""
    bcs = [O.BC_NEUMANN, O.BC_DIRICHLET, O.BC_PERIODIC]
    ns = [9, 7, 8]
    vs, lams, hs = zip(*[_mode(n, b, j) for n, b, j in zip(ns, bcs, [1, 1, 1])])
    U0 = np.multiply.outer(vs[2], np.multiply.outer(vs[1], vs[0]))[None]
    D, c, T = 0.01, -0.7, 1.0
    exact = math.exp((c - D * sum(lams)) * T)
    errs = []
    for nst in (10, 20, 40, 80):
        U = O.etd_rdp_if_run(U0, T / nst, [D], bcs, hs, "linear", {"C": [[c]]}, nst)
        errs.append(np.abs(U - exact * U0).max())
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(eoc > 1.9) and np.all(eoc < 2.2), eoc


def test_manufactured_solution_second_order_in_h_and_k():
    """u = exp(-t) cos(pi x) cos(pi y) solves u_t = D Lap u + (2 pi^2 D - 1) u
    with homogeneous Neumann conditions on the unit square."""
    D = 0.1
    c = 2 * math.pi**2 * D - 1.0
    T = 0.5
    errs = []
    for n in (9, 17, 33):
        h = 1.0 / (n - 1)
        x = np.arange(n) * h
        U0 = np.outer(np.cos(math.pi * x), np.cos(math.pi * x))[None]
        nst = n - 1
        U = O.etd_rdp_if_run(U0, T / nst, [D], [O.BC_NEUMANN] * 2, [h, h], "linear", {"C": [[c]]}, nst)
        errs.append(np.abs(U - math.exp(-T) * U0).max())
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(eoc > 1.85) and np.all(eoc < 2.3), (errs, eoc)


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------

def test_uniform_steady_states_are_fixed_points():
    n3 = (4, 5, 6)
    cases = [
        ("brusselator", {"a": 1.0, "b": 3.4}, (1.0, 3.4), O.BC_NEUMANN),
        ("gray_scott", {"F": 0.04, "kappa": 0.06}, (1.0, 0.0), O.BC_PERIODIC),
    ]
    for model, p, ss, bc in cases:
        U = np.stack([np.full(n3, ss[0]), np.full(n3, ss[1])])
        hs = [O.default_h(n, bc) for n in n3[::-1]]
        got = O.etd_rdp_if_run(U, 0.3, [0.02, 0.01], [bc] * 3, hs, model, p, 3)
        np.testing.assert_allclose(got, U, rtol=0, atol=1e-13)
    # Schnakenberg about u* = (a + b, b/(a+b)^2) with Dirichlet on w = u - u*.
    a, b = 0.1, 0.9
    p = {"a": a, "b": b, "gamma": 1.0, "shift": [a + b, b / (a + b) ** 2]}
    W = np.zeros((2,) + n3)
    got = O.etd_rdp_if_run(W, 1e-3, [1.0, 10.0], [O.BC_DIRICHLET] * 3,
                           [O.default_h(n, O.BC_DIRICHLET) for n in n3[::-1]], "schnakenberg", p, 3)
    assert np.abs(got).max() < 1e-15


def test_pure_diffusion_conserves_weighted_mass():
    rng = np.random.default_rng(4)
    U = rng.random((2, 5, 6, 7))
    k, D = 0.2, [0.05, 0.4]
    for bc in (O.BC_NEUMANN, O.BC_PERIODIC):
        hs = [O.default_h(n, bc) for n in (7, 6, 5)]
        got = O.etd_rdp_if_run(U, k, D, [bc] * 3, hs, "linear", {"C": np.zeros((2, 2))}, 4)
        wts = []
        for n in (5, 6, 7):
            w = np.ones(n)
            if bc == O.BC_NEUMANN:
                w[0] = w[-1] = 0.5
            wts.append(w)
        Wt = np.multiply.outer(wts[0], np.multiply.outer(wts[1], wts[2]))
        for s in range(2):
            assert abs((Wt * got[s]).sum() - (Wt * U[s]).sum()) < 1e-12 * (Wt * U[s]).sum()


def test_axes_below_d_commute_and_axis_d_does_not():
    rng = np.random.default_rng(5)
    U = 0.5 + 0.2 * rng.random((2, 6, 5, 7))  # n1 = 7, n2 = 5, n3 = 6
    bcs = [O.BC_NEUMANN, O.BC_DIRICHLET, O.BC_PERIODIC]
    hs = [0.11, 0.13, 0.17]
    p = {"F": 0.04, "kappa": 0.06}
    k, D = 0.5, [0.02, 0.01]
    ref = O.etd_rdp_if_step(U, k, D, bcs, hs, "gray_scott", p)
    # Swap axes 1 and 2: same result, transposed.
    Us = np.swapaxes(U, 2, 3)
    got = O.etd_rdp_if_step(Us, k, D, [bcs[1], bcs[0], bcs[2]], [hs[1], hs[0], hs[2]], "gray_scott", p)
    np.testing.assert_allclose(np.swapaxes(got, 2, 3), ref, rtol=1e-13, atol=1e-14)
    # Swapping axis 1 with axis d changes the scheme (it is not symmetric in d).
    Uz = np.swapaxes(U, 1, 3)
    got = O.etd_rdp_if_step(Uz, k, D, [bcs[2], bcs[1], bcs[0]], [hs[2], hs[1], hs[0]], "gray_scott", p)
    assert np.abs(np.swapaxes(got, 1, 3) - ref).max() > 1e-9


def test_reflection_equivariance():
    rng = np.random.default_rng(6)
    U = rng.random((2, 5, 6, 7))
    bcs = [O.BC_NEUMANN, O.BC_DIRICHLET, O.BC_PERIODIC]
    hs = [0.1, 0.2, 0.3]
    p = {"a": 1.0, "b": 3.0}
    ref = O.etd_rdp_if_step(U, 0.1, [0.1, 0.2], bcs, hs, "brusselator", p)
    for ax in (1, 2, 3):
        got = O.etd_rdp_if_step(np.flip(U, ax), 0.1, [0.1, 0.2], bcs, hs, "brusselator", p)
        np.testing.assert_allclose(np.flip(got, ax), ref, rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------------------
# Paper experiments at small scale
# ---------------------------------------------------------------------------

def test_brusselator_2d_observed_order_two():
    """Section 8.2 setup (Neumann, D = 2e-3, A = 3.4, B = 1, u1 = 1/2 + y,
    u2 = 1 + 5x) on a coarse grid: the error against a fine-k run of the same
    space discretisation decays at order about two (Table brutable)."""
    n = 21
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")  # array axis 0 is y (axis 2)
    U0 = np.stack([0.5 + Y, 1.0 + 5.0 * X])
    p = {"a": 1.0, "b": 3.4}  # paper's B = 1 is a, A = 3.4 is b
    T = 2.0
    args = ([2e-3, 2e-3], [O.BC_NEUMANN] * 2, [h, h], "brusselator", p)
    ref = O.etd_rdp_if_run(U0, T / 2560, *args, 2560)
    errs = []
    for nst in (40, 80, 160):
        errs.append(np.abs(O.etd_rdp_if_run(U0, T / nst, *args, nst) - ref).max())
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    lo = min(GOLD["brusselator_eoc_etd_rdp_if"]["value"]) - 0.15
    hi = max(GOLD["brusselator_eoc_etd_rdp_if"]["value"]) + 0.05
    assert np.all(eoc > lo) and np.all(eoc < hi), eoc


def test_enzyme_2d_observed_order_two():
    """Section 8.1 (Table enztable): enzyme kinetics on the unit square,
    homogeneous Dirichlet, D = 0.2, h = 0.0125 (79 interior points), initial
    value one, T = 1, k = 0.05 ... 0.00625.  The error against a fine-k run of
    the same space discretisation decays at the printed order (the printed
    errors themselves depend on a reference solution the paper does not
    state)."""
    n = 79
    h = 1.0 / (n + 1)
    assert abs(h - 0.0125) < 1e-15
    U0 = np.ones((1, n, n))
    args = ([0.2], [O.BC_DIRICHLET] * 2, [h, h], "enzyme", {})
    ref = O.etd_rdp_if_run(U0, 1.0 / 1280, *args, 1280)
    errs = [np.abs(O.etd_rdp_if_run(U0, 1.0 / nst, *args, nst) - ref).max()
            for nst in (20, 40, 80, 160)]
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    lo = min(GOLD["enzyme_eoc_etd_rdp_if"]["value"]) - 0.15
    hi = max(GOLD["enzyme_eoc_etd_rdp_if"]["value"]) + 0.05
    assert np.all(eoc > lo) and np.all(eoc < hi), eoc
    # the solution decays (f = -u/(1+u) < 0 for u > 0) and stays positive
    assert 0.0 < ref.min() and ref.max() < 1.0


def test_brusselator_3d_approaches_printed_limit():
    """Section 8.2, 3-D Brusselator (A = 1, B = 2): the state approaches
    (B, A/B) = (2, 0.5).  Run the printed grid with a larger k to t = 20."""
    g = GOLD["brusselator_3d_limit"]["value"]
    s = GOLD["brusselator_3d_setup"]["value"]
    n = s["p"]
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    U0 = np.stack([1 + np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y) * np.sin(2 * np.pi * Z),
                   np.full(X.shape, 3.0)])
    p = {"a": g["B"], "b": g["A"]}
    U = O.etd_rdp_if_run(U0, 0.05, [s["D"]] * 2, [O.BC_NEUMANN] * 3, [h] * 3, "brusselator", p, 400)
    assert abs(U[0].mean() - g["u1"]) < 1e-3 and abs(U[1].mean() - g["u2"]) < 1e-3
    assert np.abs(U[0] - g["u1"]).max() < 5e-3
