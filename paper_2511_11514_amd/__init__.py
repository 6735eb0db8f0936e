"""Coverage-flow library for AMD MI355X (gfx950).

Python binding of libct.so (see include/ct.h): argument marshalling only, every
step of the flow evaluation runs in the library's HIP kernels.  PyTorch is used
for device memory and streams.
"""
from ._lib import (CT_DEBIAS, CT_GRAD_W, CT_VALUE, CT_WARM_START, CT_REF_CACHED,  # noqa: F401
                   CT_SAFE_LSE, CT_DYN_DOUBLE_INTEGRATOR, CT_DYN_UNICYCLE, CT_FLOW_SINKHORN,
                   CT_FLOW_SVGD, CT_FLOW_SVGD_GRID, CtError, SinkhornOpts, GMMDesc, GridDesc,
                   lib)
from .api import (sinkhorn_grad, sinkhorn_grad_batched, SinkhornDivergence, BatchedSinkhorn,  # noqa: F401
                  sinkhorn_divergence, svgd_grad, lqr_track, plan, plan_ensemble,
                  autotune_sinkhorn,
                  tuning_table, tuning_save, tuning_load, tuning_clear, GMM, version,
                  probe_alu_rates, svgd_grad_score, UtilityGrid, grid_score, grid_samples,
                  reference_self_potential, static_scratch_bytes)

__version__ = "0.1.0"
