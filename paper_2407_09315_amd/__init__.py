"""MI355X (gfx950) random batch Ewald k-space force: HIP library + thin Python binding."""
from .rbe import (Batch, Plan, RBEError, rbe_evaluate, rbe_evaluate_static, rbe_ewald_weights, rbe_kspace_force,  # noqa: F401
                  rbe_kspace_virial, rbe_kspace_vjp, rbe_normalization, rbe_plan_upload, rbe_sample_k, rbe_sample_k_metropolis,
                  rbe_sample_k_device, rbe_structure_factor, RBLPlan, rbl_short_force)
from .autograd import RBEKSpace, rbe_kspace  # noqa: F401
