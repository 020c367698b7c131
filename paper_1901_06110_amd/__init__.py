"""MI355X (gfx950) DSG-NLM denoiser and linearized plug-and-play ADMM.

Thin Python layer over the C ABI of libdsnlm.so (include/dsnlm.h): it passes
torch CUDA tensors' device pointers and the current HIP stream.  Every step of
the computation runs in the library's HIP kernels; importing the binding fails
if the library has not been built.
"""
from __future__ import annotations

from .api import (  # noqa: F401
    Weights,
    dsnlm_apply,
    dsnlm_apply_backward,
    dsnlm_build_weights,
    dsnlm_forward,
    dsnlm_forward_batched,
    dsnlm_nlm,
    dsnlm_forward_brute,
    dsnlm_backward_batched,
    dsnlm_batched_state,
    ladmm_apply_forward,
    ladmm_gradient,
    ladmm_operator_norm2,
    ladmm_solve,
    ladmm_solve_backward,
    admm_cg_solve,
    ladmm_step,
    SROperator,
    SPIOperator,
    LadmmParams,
)

from .autograd import DSNLMFunction, UnrolledLADMM, dsnlm, unrolled_ladmm  # noqa: F401,E402

__version__ = "0.1.0"
