"""FP64 CPU oracle for the coverage-flow hot path.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package.  It shares no code
with the HIP path (neither imports the other); the only common dependency is
the seeded input generator module ``workloads``.

Each function follows the paper's definitions directly, in float64:

* ``sinkhorn``   - debiased Sinkhorn divergence, its gradient with respect to
                   the trajectory samples and the reference weights
                   (Sec. II-B, eqs. 5-7);
* ``gmm_score``, ``median_bandwidth`` (and ``median_bandwidth_by_counting``
                   for large n), ``svgd_phi`` - the Stein variational
                   flow with an RBF kernel and an analytic mixture score
                   (Sec. II-B, eq. 4);
* ``grid``       - a reference given as a utility on a grid: its score for the
                   Stein flow and its weighted nodes for the Sinkhorn flow
                   (Sec. II-A, Sec. II-B);
* ``lqr_track_dense``, ``lqr_track_riccati`` - linear-quadratic flow matching
                   (Sec. II-C, eqs. 8-10);
* ``plan_step`` / ``plan`` - the outer planning loop (Sec. II-C).
"""
from .sinkhorn import sinkhorn, lse_update, gauge_fix, SinkhornResult  # noqa: F401
from .svgd import (gmm_score, gmm_logpdf, median_bandwidth, median_bandwidth_by_counting,  # noqa: F401
                   svgd_phi, pair_count)
from . import grid  # noqa: F401
from .lqr import lqr_track_dense, lqr_track_riccati  # noqa: F401
from .plan import (dynamics_f, dynamics_jac, rollout, plan_step, plan,  # noqa: F401
                   reference_flow)
