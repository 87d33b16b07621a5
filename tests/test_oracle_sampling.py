"""The sampled full-size reference used by the GPU tests equals the oracle's
full step (checked on a small grid, CPU only)."""

import numpy as np

import oracle as O
from tests.test_gpu_parity import P, _sampled_step_reference, oracle_run


def test_oracle_sampling_equals_full_step():
    for bcs in (("periodic", "neumann", "dirichlet"), ("dirichlet", "periodic", "neumann")):
        prob = P((12, 10, 8), bcs, model="gray_scott", params={"F": 0.04, "kappa": 0.06})
        u0 = prob.initial()
        full = oracle_run(prob, u0, 1)
        x0s = [0, 5, 11]
        np.testing.assert_allclose(_sampled_step_reference(prob, u0, x0s), full[..., x0s],
                                   rtol=1e-14, atol=1e-15)
