"""FP64 CPU oracle for DSG-NLM and linearized plug-and-play ADMM.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
CPU-baseline leg may import this package.  It shares no code with the HIP
library (paper_1901_06110_amd) and imports nothing from it; the only module
both sides read is `synth`, which draws the seeded inputs.

Modules
-------
dsnlm_ref  -- the doubly stochastic NLM denoiser (Section 3, eqs. NLM, S1-S3,
              Algorithm 2), two independent routes.
ladmm_ref  -- forward models (Section 4.1 eq. dataterm, Section 4.2 eqs. obj and
              photongrad) and Algorithm 1 (Section 2).
grad_ref   -- finite-difference and FP64-autograd reference gradients.

Every function in these modules is pinned by a CPU test against something
other than itself (closed forms, invariants, brute force on tiny inputs,
library routines); the ones that are not say "parity unpinned".
"""
