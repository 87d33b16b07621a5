"""Point values of the oracle's reaction terms, Jacobians and parameter
derivatives against numbers worked out by hand from the model formulas.

The models: Michaelis-Menten enzyme kinetics f = -u/(1+u) (Section 8.1), the
Brusselator (Section 8.2; the benchmark's a, b are the paper's B, A), the
complex Ginzburg-Landau term u - (1 + i beta) u |u|^2 (Section 8.3), the cubic
Schroedinger term -i (B + C |u|^2) u (Section 8.4), and the two benchmark
systems that are not in the paper, Gray-Scott
(-u v^2 + F (1 - u), u v^2 - (F + kappa) v) and Schnakenberg
(gamma (a - u + u^2 v), gamma (b - u^2 v)).

The evaluation point (u, v) = (0.3, 0.7) is far from every steady state, and
gamma = 2, so that each term shows: swapping u v^2 for u^2 v, dropping gamma,
flipping a sign or a parameter changes a value by far more than the
tolerance.  Arithmetic used below:
    u^2 = 0.09, v^2 = 0.49, u v = 0.21, u^2 v = 0.063, u v^2 = 0.147,
    u^2 + v^2 = 0.58.
"""

import numpy as np
import pytest

import oracle as O

U0, V0 = 0.3, 0.7


def _pt(*vals):
    """A 2-species state of one cell (shape (s, 1))."""
    return np.array(vals, dtype=np.float64).reshape(len(vals), 1)


# (model, params, f, J (row i = dF_i), dF/dtheta per parameter in
#  param_names order)
CASES = [
    (
        "enzyme", {},
        # f = -0.3/1.3 = -3/13;  J = -1/(1.3)^2 = -100/169
        [-3.0 / 13.0],
        [[-100.0 / 169.0]],
        [],
    ),
    (
        "brusselator", {"a": 1.0, "b": 3.4},
        # f0 = 1 - 4.4*0.3 + 0.063 = -0.257;  f1 = 3.4*0.3 - 0.063 = 0.957
        [-0.257, 0.957],
        # [[-(b+1) + 2uv, u^2], [b - 2uv, -u^2]]
        [[-3.98, 0.09], [2.98, -0.09]],
        # d/da = (1, 0);  d/db = (-u, u)
        [[1.0, 0.0], [-0.3, 0.3]],
    ),
    (
        "gray_scott", {"F": 0.04, "kappa": 0.06},
        # f0 = -0.147 + 0.04*0.7 = -0.119;  f1 = 0.147 - 0.10*0.7 = 0.077
        [-0.119, 0.077],
        # [[-v^2 - F, -2uv], [v^2, 2uv - (F + kappa)]]
        [[-0.53, -0.42], [0.49, 0.32]],
        # d/dF = (1 - u, -v);  d/dkappa = (0, -v)
        [[0.7, -0.7], [0.0, -0.7]],
    ),
    (
        "schnakenberg", {"a": 0.1, "b": 0.9, "gamma": 2.0},
        # f0 = 2 (0.1 - 0.3 + 0.063) = -0.274;  f1 = 2 (0.9 - 0.063) = 1.674
        [-0.274, 1.674],
        # gamma [[-1 + 2uv, u^2], [-2uv, -u^2]]
        [[-1.16, 0.18], [-0.84, -0.18]],
        # d/da = (gamma, 0);  d/db = (0, gamma);  d/dgamma = (a - u + u^2 v, b - u^2 v)
        [[2.0, 0.0], [0.0, 2.0], [-0.137, 0.837]],
    ),
    (
        "cgl", {"beta": 1.3},
        # (p, q) = (Re u, Im u) = (0.3, 0.7):  (1 + 1.3i)(0.3 + 0.7i) = -0.61 + 1.09i,
        # times |u|^2 = 0.58: -0.3538 + 0.6322i;  u minus that = 0.6538 + 0.0678i
        [0.6538, 0.0678],
        # f0 = p - (p - beta q) m2, f1 = q - (q + beta p) m2, m2 = p^2 + q^2:
        # df0/dp = 1 - m2 - 2p (p - beta q) = 0.42 + 0.366 = 0.786
        # df0/dq = beta m2 - 2q (p - beta q) = 0.754 + 0.854 = 1.608
        # df1/dp = -beta m2 - 2p (q + beta p) = -0.754 - 0.654 = -1.408
        # df1/dq = 1 - m2 - 2q (q + beta p) = 0.42 - 1.526 = -1.106
        [[0.786, 1.608], [-1.408, -1.106]],
        # d/dbeta = (q m2, -p m2) = (0.406, -0.174)
        [[0.406, -0.174]],
    ),
    (
        "linear", {"C": [[-0.3, 0.2], [0.1, -0.5]]},
        # C u: (-0.09 + 0.14, 0.03 - 0.35)
        [0.05, -0.32],
        [[-0.3, 0.2], [0.1, -0.5]],
        # d/dC_ij = u_j e_i, row-major
        [[0.3, 0.0], [0.7, 0.0], [0.0, 0.3], [0.0, 0.7]],
    ),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_reaction_point_values(case):
    model, params, f_ref, J_ref, dth_ref = case
    s = len(f_ref)
    U = _pt(U0, V0)[:s]
    f = O.reaction(model, params, U)[:, 0]
    np.testing.assert_allclose(f, f_ref, rtol=1e-13, atol=1e-15)
    J = np.array([[float(np.ravel(J_ij)[0]) for J_ij in row]
                  for row in O.reaction_jacobian(model, params, U)])
    np.testing.assert_allclose(J, J_ref, rtol=1e-13, atol=1e-15)
    dth = [g[:, 0] for g in O.reaction_param_grads(model, params, U)]
    assert len(dth) == len(O.param_names(model, s)) == len(dth_ref)
    for got, ref in zip(dth, dth_ref):
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-15)


def test_shift_evaluates_at_the_shifted_state():
    # Schnakenberg with Dirichlet on w = u - u*: F is evaluated at w + shift.
    p = {"a": 0.1, "b": 0.9, "gamma": 2.0, "shift": [1.0, 0.9]}
    W = _pt(U0 - 1.0, V0 - 0.9)
    np.testing.assert_allclose(O.reaction("schnakenberg", p, W)[:, 0], [-0.274, 1.674],
                               rtol=1e-13)
    J = O.reaction_jacobian("schnakenberg", p, W)
    np.testing.assert_allclose([[J[0][0][0], J[0][1][0]], [J[1][0][0], J[1][1][0]]],
                               [[-1.16, 0.18], [-0.84, -0.18]], rtol=1e-13)
    dth = O.reaction_param_grads("schnakenberg", p, W)
    np.testing.assert_allclose(dth[2][:, 0], [-0.137, 0.837], rtol=1e-13)


def test_complex_species_point_values():
    u = np.array([[U0 + 1j * V0]])
    # Ginzburg-Landau with alpha in D: u - (1 + i beta) u |u|^2 (as above)
    np.testing.assert_allclose(O.reaction("cgl_z", {"beta": 1.3}, u)[0, 0], 0.6538 + 0.0678j,
                               rtol=1e-13)
    # Schroedinger: -i q u, q = B + C |u|^2 = 0.5 - 0.58 = -0.08;
    # -i (-0.08)(0.3 + 0.7i) = 0.08i (0.3 + 0.7i) = -0.056 + 0.024i
    np.testing.assert_allclose(O.reaction("nls_z", {"B": 0.5, "C": -1.0}, u)[0, 0],
                               -0.056 + 0.024j, rtol=1e-13)
    # with a per-cell field b = 0.2: q = -0.08 + 0.2 = 0.12;
    # -i (0.12)(0.3 + 0.7i) = 0.084 - 0.036i
    np.testing.assert_allclose(
        O.reaction("nls_z", {"B": 0.5, "C": -1.0, "Bfield": np.array([[0.2]])[0]}, u)[0, 0],
        0.084 - 0.036j, rtol=1e-13)
