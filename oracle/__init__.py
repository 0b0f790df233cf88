"""CPU oracle for the Gaussian kernel ridge regression hot path — TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 NumPy/SciPy code written from the paper (arXiv 1905.10587,
"Fast and Accurate Gaussian Kernel Ridge Regression Using Matrix Decompositions
for Preconditioning").  It is the checker the HIP library is compared against,
not a fallback: only the test suite, the smoke entry point and the benchmark's
CPU-baseline leg may import it.  It shares no code with the HIP path; both are
fed the same inputs by the separate ``datagen`` module.

Modules
  kernel   Gaussian kernel matrix, matrix-free kernel MVM, derivative kernel (Sec. 1, Eq. 1-2, Eq. dscrt_gt)
  precond  Algorithms 1-4: sketches, pivoted QR anchor selection, Nystrom factor, Woodbury apply (Sec. 3);
           farthest point sampling and caller-given anchors (remark in Sec. 3)
  pcg      Algorithm 5: preconditioned CG with residual replacement and Lanczos estimates (Sec. 3, 4.1)
  adjoint  validation-loss gradient w.r.t. log eps and log beta (adjoint method; not in the paper)
  theory   Theorem maintheorem, the ID corollary, the SVD remark, Corollary tradeoff (also on a dataset's
           bounding box), CG rate (Sec. 4)

Parity status: every function is pinned by the CPU tests in tests/test_oracle_*.py
except the FP32 / mixed-precision error levels of the GPU path, which have no
closed form (parity unpinned beyond the error bounds stated with each test).
"""
from . import kernel, precond, pcg, adjoint, theory  # noqa: F401
