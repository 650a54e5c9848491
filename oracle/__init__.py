"""Plain FP64 CPU oracle for the TT-UTV hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only the tests, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the HIP library.
"""
from .ttutv_oracle import (  # noqa: F401
    sketch_gaussian, splitmix64, tt_utv, tt_svd, tt_reconstruct, tt_sample,
    tt_sample_grad, step_tall_view, canonical_signs, completion_step,
    left_orthogonalize, right_orthogonalize, tt_sample_grad_mixed, riemannian_gradient, tangent_train,
    rgrad_step, tt_reconstruct_grad,
)
