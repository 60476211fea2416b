"""MI355X-native Wilson-Dirac multi-mass BiCGstab (HIP kernels behind the C ABI of libwdirac.so).

Paper: Alexandru, Pelissier, Gamari, Lee, "Multi-mass solvers for lattice QCD on GPUs".
"""
from ._lib import (  # noqa: F401
    EXPORTED, Gauge, OpVariant, SolverParams, SolverStats, WdError, bicgstab_m_solve, bicgstab_solve, load,
    op_variant, params, set_graphs, timing_enable, timing_get, timing_reset, wd_apply, wd_apply_dag, wd_apply_noalloc,
    wd_apply_prec, wd_batch_solve, wd_gauge_create,
    wd_gauge_destroy, wd_gauge_grad, wd_multimass_solve, wd_normal_solve, WD_METHOD_BATCHED, WD_METHOD_MULTISHIFT,
    WD_METHOD_SEQUENTIAL, WD_GUESS_NONE, WD_GUESS_POLY, WD_GUESS_MINRES, WD_MIXED_DEFECT, WD_MIXED_RELIABLE, LIBPATH,
)
from .autograd import WilsonSolve, wilson_solve  # noqa: F401
