"""FP64 CPU oracle for the sparse-coding hot path -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library (the HIP path and its binding)
neither imports nor calls it, and the two share no code.

Contents:
  omp, sh_basis, radiance    -- ctypes wrappers over sc_oracle.c (plain C, FP64)
  mlp_*                      -- the support-proposer network in NumPy FP64
  restricted/learned pursuit -- the proposer-guided encoder, step by step
  mod_learn                  -- dictionary learning by alternating minimisation
  pack_csc, gaussian_rgb     -- CSC storage of the codes, per-Gaussian colour
"""
from .core import (  # noqa: F401
    build,
    lib_path,
    omp,
    omp_restricted,
    sh_basis,
    radiance,
    gram,
)
from .mlp import (  # noqa: F401
    gelu,
    gelu_grad,
    mlp_forward,
    mlp_loss_and_grads,
    bce_with_logits,
    adam_step,
    topk_lowest_index,
    bf16_round,
    multi_hot,
)
from .learned import learned_encode  # noqa: F401
from .dictlearn import mod_learn, mod_step  # noqa: F401
from .csc import SH_C0, pack_csc, unpack_csc, gaussian_rgb  # noqa: F401
