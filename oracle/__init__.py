"""FP64 CPU oracle for the ETD-RDP-IF scheme (Asante-Asamani, Kleefeld, Wade).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The GPU library never imports it, shares no code, table or helper
with it, and must fail loudly rather than fall back to it.

The oracle is plain and slow on purpose: dense or LAPACK banded line solves,
an FFT for the periodic circulant systems, and the scheme's formulas written
out in the order the paper gives them.  See ``etd_rdp_oracle`` for the
citations of each function.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against values the paper or the mathematics fix (closed forms, eigenvector
expansions, dense Kronecker brute force, reaction values worked out by hand,
Heun reduction, invariants, observed convergence order against the printed
orders, central differences for the reverse mode).
"""

from .etd_rdp_oracle import (  # noqa: F401
    BC_DIRICHLET,
    BC_NEUMANN,
    BC_PERIODIC,
    default_h,
    laplacian_matrix,
    line_matrix,
    solve_axis,
    apply_R,
    reaction,
    etd_rdp_if_step,
    etd_rdp_if_run,
    step_intermediates,
    etd1_if_step,
    r_rdp,
    adjoint_step,
    param_names,
    reaction_jacobian,
    reaction_param_grads,
    solve_axis_T,
    laplacian_axis,
)
