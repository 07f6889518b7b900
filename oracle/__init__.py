"""Plain, slow, FP64 CPU oracle for the RBF-FD stencil hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it.  It
shares no code with the GPU path: the only common module is ``nodesets`` (seeded
geometry, none of the method's arithmetic).

Contents, each following the paper's definitions (Slak & Kosec, "Medusa",
Sec. 2.1 and 2.2.2):

* ``knn``     -- stencil selection: the n_i closest nodes, self first (Sec. 2.1).
* ``rbffd``   -- RBF-FD weights from the augmented system, eq. (rbf-system-aug).
* ``csr``     -- the sparse operator with at most sum(n_i) nonzeros (Sec. 2.3.2).
* ``refine``  -- FP32 LU + FP64-residual iterative refinement, used to predict
                 which stencils the mixed-precision form must send to FP64.
* ``mlp``     -- the surrogate network (forward/backward/Adam) in FP64 with
                 BF16 rounding emulated at the GPU's rounding points.
* ``project`` -- projection of surrogate weights onto the polynomial
                 reproduction constraints (second block row of the system).
* ``poisson`` -- manufactured Poisson problem on the annulus (Sec. 5) and the
                 Laplacian error e_h of Sec. 3.2.
"""
from . import knn, rbffd, csr, refine, mlp, project, poisson  # noqa: F401
