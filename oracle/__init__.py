"""Plain FP64 CPU oracle for s-FairSC (test infrastructure only).

This package is the independent reference the GPU library is checked
against.  It is deliberately slow and literal: dense or scipy-sparse FP64
arithmetic, library routines (QR, eigh, eigsh, lstsq, linear_sum_assignment)
used as single steps, no blocking or fusion.  Each function names the passage
of the paper it restates.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import it.  It shares no code with the GPU library and imports nothing from it;
the product path never calls it.

Functions whose output has no pin (a check against something other than the
oracle itself) say "parity unpinned" in their docstring.  Currently every
function is pinned by a test in tests/test_oracle_*.py.
"""

from .fairsc import (  # noqa: F401
    validate_graph,
    degrees,
    laplacian,
    normalized_laplacian,
    group_indicator,
    fairness_matrix,
    constraint_matrix,
    shift_sigma,
    fair_eigs_dense,
    fair_eigs_implicit,
    fair_eigs_deflated,
    deflated_operator_dense,
    apply_deflated_operator,
    residual_norms,
)
from .kmeans import kmeans, kmeans_pp_seeds, lloyd  # noqa: F401
from .splitmix import splitmix64_outputs, splitmix64_uniform  # noqa: F401
from .metrics import (  # noqa: F401
    error_rate,
    error_rate_bruteforce,
    balance,
    average_balance,
    max_principal_angle,
    same_partition,
)
from .gradient import eigsum_edge_gradient, eigsum_edge_gradient_normalized  # noqa: F401
from .general_f import (  # noqa: F401
    membership_fairness_matrix,
    general_constraint_matrix,
    range_basis,
    fair_eigs_dense_general,
    fair_eigs_implicit_general,
    apply_deflated_operator_general,
)
from .lsqr import lsqr, project_lsqr, membership_constraint_matrix  # noqa: F401
from .ritz import ritz_pairs, krylov_schur_keep  # noqa: F401
