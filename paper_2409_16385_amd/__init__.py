"""MI355X (gfx950) contact stage of Embedded IPC (arXiv 2409.16385).

Thin Python binding over the C ABI of ``libeipc.so`` (declared in
``include/eipc.h``): argument marshalling only.  Every step of the contact
stage runs in the library's HIP kernels; PyTorch supplies device memory
and streams.  There is no CPU fallback: importing works without a GPU, but
every compute call needs the built library and a ROCm device and raises
otherwise.
"""
from .binding import (  # noqa: F401
    ENERGY, GRAD, HESS, PROJECT, MOLLIFY, SQDIST, PROJECT_REDUCED, EipcError, Context, Scene, lib_path,
    embed, build_candidates, barrier_reduce, ccd_max_step, barrier_hvp,
    narrow_phase, pair_eval, ccd_candidates, ccd_toi, fp64_selftest, bsr_to_dense,
    cholesky, cholesky_solve, Plan, StepOut, set_tuning, set_ccd_method, CCD_ADDITIVE, CCD_CLOSEST_DIRECTION,
    plan_step, contact_step, step_pairs,
    friction_lag, friction_reduce,
    reduced_mass, elastic, ELASTIC_LINEAR, ELASTIC_COROTATIONAL,
)
from .autograd import BarrierState, barrier_energy, barrier_grad  # noqa: F401
