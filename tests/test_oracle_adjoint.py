"""Pins of the oracle's reverse-mode step against central finite differences
of the oracle's forward step (the adjoint is the chain rule of the frame of
Section 6; the paper has none)."""

import numpy as np
import pytest

import oracle as O

CASES = [
    ("schnakenberg", {"a": 0.1, "b": 0.9, "gamma": 1.0}, ("neumann", "neumann", "neumann"), (1.0, 10.0), 1e-3),
    ("gray_scott", {"F": 0.04, "kappa": 0.06}, ("periodic", "dirichlet", "neumann"), (0.02, 0.01), 0.3),
    ("brusselator", {"a": 1.0, "b": 3.4}, ("neumann", "periodic"), (0.05, 0.02), 0.05),
    ("cgl", {"beta": 1.3}, ("dirichlet", "neumann", "periodic"), (0.3, 0.3), 0.05),
    ("linear", {"C": [[-0.3, 0.2], [0.1, -0.5]]}, ("neumann", "dirichlet"), (0.2, 0.05), 0.1),
    # Section 8.1's model, one species: its Jacobian -1/(1+u)^2 enters the
    # state gradient and the D gradient; it has no reaction parameters
    ("enzyme", {}, ("dirichlet", "neumann", "periodic"), (0.2,), 0.05),
]


def _setup(model, bcs, seed=0):
    rng = np.random.default_rng(seed)
    shape = (2, 4, 5, 3)[: len(bcs) + 1] if len(bcs) == 3 else (2, 5, 4)
    base = {"schnakenberg": (1.0, 0.9)}.get(model, (0.6, 0.4))
    U = np.stack([base[0] + 0.2 * rng.random(shape[1:]), base[1] + 0.2 * rng.random(shape[1:])])
    if model == "enzyme":
        U = U[:1]
    tgt = U + 0.1 * rng.standard_normal(U.shape)
    ns = U.shape[1:][::-1]
    hs = [O.default_h(n, b) for n, b in zip(ns, bcs)]
    return U, tgt, hs, rng


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_adjoint_step_matches_central_differences(case):
    model, params, bcs, D, k = case
    U, tgt, hs, rng = _setup(model, bcs)

    def loss(U_, D_, p_):
        out = O.etd_rdp_if_step(U_, k, D_, bcs, hs, model, p_)
        return float(np.sum((out - tgt) ** 2))

    out = O.etd_rdp_if_step(U, k, D, bcs, hs, model, params)
    lam = 2.0 * (out - tgt)
    gU, gD, gth = O.adjoint_step(U, lam, k, D, bcs, hs, model, params)

    eps = 1e-6
    V = rng.standard_normal(U.shape)
    fd = (loss(U + eps * V, D, params) - loss(U - eps * V, D, params)) / (2 * eps)
    assert abs(fd - np.sum(gU * V)) <= 1e-6 * max(1.0, abs(fd))

    for i in range(len(D)):
        Dp, Dm = list(D), list(D)
        h = eps * max(abs(D[i]), 1e-3)
        Dp[i] += h
        Dm[i] -= h
        fd = (loss(U, Dp, params) - loss(U, Dm, params)) / (2 * h)
        assert abs(fd - gD[i]) <= 1e-5 * max(1.0, abs(fd)), (i, fd, gD[i])

    names = O.param_names(model, U.shape[0])
    for i, nm in enumerate(names):
        if model == "linear":
            C = np.array(params["C"], dtype=float)
            Cp, Cm = C.copy(), C.copy()
            r, c = divmod(i, U.shape[0])
            Cp[r, c] += eps
            Cm[r, c] -= eps
            pp, pm = {"C": Cp}, {"C": Cm}
            h = eps
        else:
            h = eps * max(abs(params[nm]), 1e-3)
            pp, pm = dict(params), dict(params)
            pp[nm] += h
            pm[nm] -= h
        fd = (loss(U, D, pp) - loss(U, D, pm)) / (2 * h)
        assert abs(fd - gth[i]) <= 1e-5 * max(1.0, abs(fd)), (nm, fd, gth[i])


def test_shifted_reaction_adjoint():
    params = {"a": 0.1, "b": 0.9, "gamma": 1.0, "shift": [1.0, 0.9]}
    bcs = ("dirichlet",) * 3
    U, tgt, hs, rng = _setup("schnakenberg", bcs)
    U = U - np.array([1.0, 0.9]).reshape(2, 1, 1, 1)
    k, D = 1e-3, (1.0, 10.0)
    out = O.etd_rdp_if_step(U, k, D, bcs, hs, "schnakenberg", params)
    lam = 2.0 * (out - tgt)
    gU, _, _ = O.adjoint_step(U, lam, k, D, bcs, hs, "schnakenberg", params)
    V = rng.standard_normal(U.shape)
    eps = 1e-6
    lp = np.sum((O.etd_rdp_if_step(U + eps * V, k, D, bcs, hs, "schnakenberg", params) - tgt) ** 2)
    lm = np.sum((O.etd_rdp_if_step(U - eps * V, k, D, bcs, hs, "schnakenberg", params) - tgt) ** 2)
    assert abs((lp - lm) / (2 * eps) - np.sum(gU * V)) <= 1e-6 * abs(np.sum(gU * V))


def test_term_scale_bounds_every_entry():
    """The optional term-size output is the sum of |terms| of each entry: it
    bounds the entry (triangle inequality) and leaves the results unchanged."""
    model, params, bcs, D, k = CASES[1]
    U, tgt, hs, rng = _setup(model, bcs)
    lam = rng.standard_normal(U.shape)
    ts = {}
    a = O.adjoint_step(U, lam, k, D, bcs, hs, model, params)
    b = O.adjoint_step(U, lam, k, D, bcs, hs, model, params, term_scale=ts)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert np.all(np.abs(b[1]) <= ts["D"]) and np.all(ts["D"] > 0)
    assert np.all(np.abs(b[2]) <= ts["theta"]) and np.all(ts["theta"] > 0)
